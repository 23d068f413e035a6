// Dense kernels of the host factorisation: C += sign * A B^T with a register
// tile (two vectors per column of C, at least eight accumulators: enough
// independent FMA chains to cover the FMA latency on two ports), over panels
// of A and B packed 256 columns of K at a time so that the inner loop reads
// both contiguously.  Two versions: AVX2 (4-wide, 8 x 4 tiles) and, on CPUs
// that have it (checked at run time), AVX-512 (8-wide, 16 x 8 tiles).
#include "dense_host.hpp"

#include <immintrin.h>

#include <algorithm>
#include <vector>

namespace scasm {
namespace {

constexpr int kNR = 4;      // columns of C per micro-tile
constexpr int64_t kKC = 256;

// C[0:mr, 0:nr] += sign * sum_k pa[k][0:8] pb[k][0:4]; pa, pb packed (zero
// padded past mr / nr)
inline void micro_8x4(int64_t kc, const double* __restrict__ pa, const double* __restrict__ pb, double* C,
                      int64_t ldc, int mr, int nr, double sign) {
    constexpr int kMR = 8;
    __m256d c00 = _mm256_setzero_pd(), c01 = _mm256_setzero_pd();
    __m256d c10 = _mm256_setzero_pd(), c11 = _mm256_setzero_pd();
    __m256d c20 = _mm256_setzero_pd(), c21 = _mm256_setzero_pd();
    __m256d c30 = _mm256_setzero_pd(), c31 = _mm256_setzero_pd();
    for (int64_t k = 0; k < kc; ++k) {
        const __m256d a0 = _mm256_loadu_pd(pa + 8 * k);
        const __m256d a1 = _mm256_loadu_pd(pa + 8 * k + 4);
        __m256d b = _mm256_broadcast_sd(pb + 4 * k);
        c00 = _mm256_fmadd_pd(a0, b, c00);
        c01 = _mm256_fmadd_pd(a1, b, c01);
        b = _mm256_broadcast_sd(pb + 4 * k + 1);
        c10 = _mm256_fmadd_pd(a0, b, c10);
        c11 = _mm256_fmadd_pd(a1, b, c11);
        b = _mm256_broadcast_sd(pb + 4 * k + 2);
        c20 = _mm256_fmadd_pd(a0, b, c20);
        c21 = _mm256_fmadd_pd(a1, b, c21);
        b = _mm256_broadcast_sd(pb + 4 * k + 3);
        c30 = _mm256_fmadd_pd(a0, b, c30);
        c31 = _mm256_fmadd_pd(a1, b, c31);
    }
    const __m256d s = _mm256_set1_pd(sign);
    if (mr == kMR && nr == kNR) {
        double* c0 = C;
        double* c1 = C + ldc;
        double* c2 = C + 2 * ldc;
        double* c3 = C + 3 * ldc;
        _mm256_storeu_pd(c0, _mm256_fmadd_pd(s, c00, _mm256_loadu_pd(c0)));
        _mm256_storeu_pd(c0 + 4, _mm256_fmadd_pd(s, c01, _mm256_loadu_pd(c0 + 4)));
        _mm256_storeu_pd(c1, _mm256_fmadd_pd(s, c10, _mm256_loadu_pd(c1)));
        _mm256_storeu_pd(c1 + 4, _mm256_fmadd_pd(s, c11, _mm256_loadu_pd(c1 + 4)));
        _mm256_storeu_pd(c2, _mm256_fmadd_pd(s, c20, _mm256_loadu_pd(c2)));
        _mm256_storeu_pd(c2 + 4, _mm256_fmadd_pd(s, c21, _mm256_loadu_pd(c2 + 4)));
        _mm256_storeu_pd(c3, _mm256_fmadd_pd(s, c30, _mm256_loadu_pd(c3)));
        _mm256_storeu_pd(c3 + 4, _mm256_fmadd_pd(s, c31, _mm256_loadu_pd(c3 + 4)));
        return;
    }
    alignas(32) double t[kNR][kMR];
    _mm256_store_pd(&t[0][0], c00);
    _mm256_store_pd(&t[0][4], c01);
    _mm256_store_pd(&t[1][0], c10);
    _mm256_store_pd(&t[1][4], c11);
    _mm256_store_pd(&t[2][0], c20);
    _mm256_store_pd(&t[2][4], c21);
    _mm256_store_pd(&t[3][0], c30);
    _mm256_store_pd(&t[3][4], c31);
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < mr; ++i) C[i + j * ldc] += sign * t[j][i];
}

// The same with 8-wide vectors: a 16 x 8 tile (sixteen accumulators; the
// AVX-512 register file holds them with the two A vectors and a broadcast).
__attribute__((target("avx512f"))) inline void micro_16x8(int64_t kc, const double* __restrict__ pa,
                                                          const double* __restrict__ pb, double* C, int64_t ldc,
                                                          int mr, int nr, double sign) {
    constexpr int kMR = 16, kNB = 8;
    __m512d c0[kNB], c1[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
        c0[j] = _mm512_setzero_pd();
        c1[j] = _mm512_setzero_pd();
    }
    for (int64_t k = 0; k < kc; ++k) {
        const __m512d a0 = _mm512_loadu_pd(pa + 16 * k);
        const __m512d a1 = _mm512_loadu_pd(pa + 16 * k + 8);
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            const __m512d b = _mm512_set1_pd(pb[kNB * k + j]);
            c0[j] = _mm512_fmadd_pd(a0, b, c0[j]);
            c1[j] = _mm512_fmadd_pd(a1, b, c1[j]);
        }
    }
    const __m512d s = _mm512_set1_pd(sign);
    if (mr == kMR && nr == kNB) {
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            double* cj = C + j * ldc;
            _mm512_storeu_pd(cj, _mm512_fmadd_pd(s, c0[j], _mm512_loadu_pd(cj)));
            _mm512_storeu_pd(cj + 8, _mm512_fmadd_pd(s, c1[j], _mm512_loadu_pd(cj + 8)));
        }
        return;
    }
    alignas(64) double t[kNB][kMR];
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
        _mm512_store_pd(&t[j][0], c0[j]);
        _mm512_store_pd(&t[j][8], c1[j]);
    }
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < mr; ++i) C[i + j * ldc] += sign * t[j][i];
}

// Packed panels: B per block of kNR columns, k-major (kNR values per k); A
// per block of MR rows, k-major (MR values per k), full blocks copied with
// whole-vector moves.
template <int NR>
inline void pack_b(const double* B, int64_t ldb, int64_t N, int64_t k0, int64_t kc, double* pb) {
    const int64_t nblk = (N + NR - 1) / NR;
    for (int64_t jb = 0; jb < nblk; ++jb) {
        double* dst = pb + jb * NR * kc;
        const int64_t j0 = jb * NR;
        const int nr = (int)std::min<int64_t>(NR, N - j0);
        for (int64_t k = 0; k < kc; ++k) {
            const double* src = B + j0 + (k0 + k) * ldb;
            int jj = 0;
            for (; jj < nr; ++jj) dst[k * NR + jj] = src[jj];
            for (; jj < NR; ++jj) dst[k * NR + jj] = 0.0;
        }
    }
}

template <int MR>
inline void pack_a(const double* A, int64_t lda, int mr, int64_t i0, int64_t k0, int64_t kc, double* dst) {
    if (mr == MR) {
        for (int64_t k = 0; k < kc; ++k) {
            const double* src = A + i0 + (k0 + k) * lda;
            for (int ii = 0; ii < MR; ++ii) dst[k * MR + ii] = src[ii];
        }
        return;
    }
    for (int64_t k = 0; k < kc; ++k) {
        const double* src = A + i0 + (k0 + k) * lda;
        int ii = 0;
        for (; ii < mr; ++ii) dst[k * MR + ii] = src[ii];
        for (; ii < MR; ++ii) dst[k * MR + ii] = 0.0;
    }
}

void gemm_blocked_avx2(int64_t M, int64_t N, int64_t K, double sign, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double* C, int64_t ldc) {
    constexpr int kMR = 8;
    thread_local std::vector<double> pa, pb;
    const int64_t nblk = (N + kNR - 1) / kNR;
    pa.resize((size_t)kMR * kKC);
    pb.resize((size_t)nblk * kNR * kKC);
    for (int64_t k0 = 0; k0 < K; k0 += kKC) {
        const int64_t kc = std::min(kKC, K - k0);
        pack_b<kNR>(B, ldb, N, k0, kc, pb.data());
        for (int64_t i0 = 0; i0 < M; i0 += kMR) {
            const int mr = (int)std::min<int64_t>(kMR, M - i0);
            pack_a<kMR>(A, lda, mr, i0, k0, kc, pa.data());
            for (int64_t jb = 0; jb < nblk; ++jb) {
                const int64_t j0 = jb * kNR;
                const int nr = (int)std::min<int64_t>(kNR, N - j0);
                micro_8x4(kc, pa.data(), pb.data() + jb * kNR * kc, C + i0 + j0 * ldc, ldc, mr, nr, sign);
            }
        }
    }
}

__attribute__((target("avx512f"))) void gemm_blocked_avx512(int64_t M, int64_t N, int64_t K, double sign,
                                                            const double* A, int64_t lda, const double* B,
                                                            int64_t ldb, double* C, int64_t ldc) {
    constexpr int kMR = 16, kNB = 8;
    thread_local std::vector<double> pa, pb;
    const int64_t nblk = (N + kNB - 1) / kNB;
    pa.resize((size_t)kMR * kKC);
    pb.resize((size_t)nblk * kNB * kKC);
    for (int64_t k0 = 0; k0 < K; k0 += kKC) {
        const int64_t kc = std::min(kKC, K - k0);
        pack_b<kNB>(B, ldb, N, k0, kc, pb.data());
        for (int64_t i0 = 0; i0 < M; i0 += kMR) {
            const int mr = (int)std::min<int64_t>(kMR, M - i0);
            pack_a<kMR>(A, lda, mr, i0, k0, kc, pa.data());
            for (int64_t jb = 0; jb < nblk; ++jb) {
                const int64_t j0 = jb * kNB;
                const int nr = (int)std::min<int64_t>(kNB, N - j0);
                micro_16x8(kc, pa.data(), pb.data() + jb * kNB * kc, C + i0 + j0 * ldc, ldc, mr, nr, sign);
            }
        }
    }
}

const bool g_avx512 = __builtin_cpu_supports("avx512f");

}  // namespace

void gemm_nt(int64_t M, int64_t N, int64_t K, double sign, const double* A, int64_t lda, const double* B,
             int64_t ldb, double* C, int64_t ldc) {
    if (M <= 0 || N <= 0 || K <= 0) return;
    if (M * N * K < 4096 || K < 4) {
        for (int64_t j = 0; j < N; ++j) {
            double* c = C + j * ldc;
            for (int64_t k = 0; k < K; ++k) {
                const double b = sign * B[j + k * ldb];
                const double* a = A + k * lda;
                for (int64_t i = 0; i < M; ++i) c[i] += a[i] * b;
            }
        }
        return;
    }
    if (g_avx512) gemm_blocked_avx512(M, N, K, sign, A, lda, B, ldb, C, ldc);
    else gemm_blocked_avx2(M, N, K, sign, A, lda, B, ldb, C, ldc);
}

}  // namespace scasm
