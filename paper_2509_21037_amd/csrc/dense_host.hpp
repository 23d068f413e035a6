// Dense kernels of the host factorisation (x86-64 with AVX2 + FMA; AVX-512
// where the CPU has it, chosen at run time).
#pragma once
#include <cstdint>

namespace scasm {

// C += sign * A * B^T, column-major: A is M x K (lda), B is N x K (ldb), C is
// M x N (ldc); sign is +1 or -1.  Register-blocked 8 x 4 (AVX2) or 16 x 8
// (AVX-512) micro-kernel over packed panels of 256 columns of K; small
// products take a plain loop.
void gemm_nt(int64_t M, int64_t N, int64_t K, double sign, const double* A, int64_t lda, const double* B,
             int64_t ldb, double* C, int64_t ldc);

}  // namespace scasm
