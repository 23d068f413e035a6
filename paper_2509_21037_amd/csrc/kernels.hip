// HIP kernels for gfx950 (CDNA4, wave64): staircase TRSM and SYRK of the
// dual Schur-complement assembly (paper, Sec. 3.2 and 3.3), FP64 path.
//
// MFMA operand layouts used throughout (v_mfma_f64_16x16x4f64):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   C/D (16x16): lane l, register r holds D[4 r + l / 16][l % 16]
// so the D registers of a 16 x 16 tile are, register r, exactly the B operand
// of k-slice r of the same tile used as a right-hand side.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace scasm {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Orders this wavefront's LDS and global accesses across lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Staircase TRSM, X = L^{-1} P B^T (Sec. 3.2, factor splitting with pruning).
// One workgroup = one 64-column tile of one subdomain; wavefront w owns the
// 16-column stripe w.  The four wavefronts walk the factor blocks together,
// from the block holding the tile's first pivot (rows above it are zero and
// stay zero: forward substitution only propagates downwards); a stripe whose
// first pivot lies further down joins at its own first block.  Per block:
//   1. the dense diagonal block (<= 64 x 64) is staged in LDS once for the
//      workgroup; each wavefront loads its stripe's block rows into registers
//      (MFMA accumulator layout);
//   2. diagonal solve in FP64: 16-row sub-blocks by substitution (scaling by
//      the reciprocal of the diagonal, column-wise elimination), each followed
//      by an MFMA update of the sub-blocks below it inside the diagonal block;
//   3. the solved rows are stored, then the pruned rows below the block are
//      updated in chunks of 64, X[R_b] -= L[R_b, b] X[b], with FP64 MFMA:
//      each chunk of the factor panel is loaded once into LDS for all four
//      wavefronts (the next chunk is prefetched into registers meanwhile).
// ---------------------------------------------------------------------------
constexpr int kLdsLd = 64 + 2;            // LDS leading dimension (doubles) of a staged chunk

// Loads rows [r0, r0 + 64) x columns [0, w) of a column-major panel (leading
// dimension ld, nrows valid rows) into 16 registers per thread, negated when
// `neg` (the update subtracts).
__device__ __forceinline__ void load_chunk(const double* __restrict__ panel, int ld, int nrows, int w,
                                           int r0, bool neg, double (&reg)[16]) {
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int row = e & 63;
        const int k = e >> 6;
        const int gr = r0 + row;
        double v = 0.0;
        if (k < w && gr < nrows) v = panel[(int64_t)k * ld + gr];
        reg[it] = neg ? -v : v;
    }
}

__device__ __forceinline__ void store_chunk(double* __restrict__ sL, const double (&reg)[16]) {
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int e = threadIdx.x + 256 * it;
        sL[(e >> 6) * kLdsLd + (e & 63)] = reg[it];
    }
}

__global__ __launch_bounds__(256) void trsm_stair_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows,
    const double* __restrict__ lval, const int32_t* __restrict__ piv,
    const int8_t* __restrict__ sgn, double* __restrict__ X)
{
    __shared__ double sL[64 * kLdsLd];
    __shared__ double sRd[64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const TileDev T = tiles[blockIdx.x];
    const SubDev S = subs[T.sub];
    const int n = S.n;
    const int kstart = T.kstart;
    double* __restrict__ Xs = X + T.x_off;
    const int col = wv * kStripe + j;
    const int64_t cbase = S.col_off + (int64_t)T.tile * kTile;

    // initial right-hand side: zero trapezoid, sign at the pivot row
    const int nrows = n - kstart;
    for (int r = g; r < nrows; r += 4) Xs[(int64_t)r * kTile + col] = 0.0;
    __threadfence_block();
    if (g == 0 && col < T.ncols)
        Xs[(int64_t)(piv[cbase + col] - kstart) * kTile + col] = (double)sgn[cbase + col];
    __syncthreads();

    const BlockDev* __restrict__ B = blocks + S.blk_off;
    const int32_t* __restrict__ R = rows + S.rows_off;
    const double* __restrict__ L = lval + S.lval_off;
    const int my_start = tiles[blockIdx.x].start_block[wv];
    const int first_block = tiles[blockIdx.x].start_block[0];

    double pre[16];
    for (int b = first_block; b < S.nblocks; ++b) {
        const BlockDev bd = B[b];
        const int w = bd.w;
        const int ld = bd.ld;
        const int row0 = bd.row0;
        const int nb = bd.nbelow;
        const double* __restrict__ Lb = L + bd.lval_off;
        const bool act = b >= my_start;

        // ---- stage the diagonal block (rows [0, w) of the panel)
        load_chunk(Lb, ld, w, w, 0, false, pre);
        __syncthreads();                 // previous users of sL are done
        store_chunk(sL, pre);
        __syncthreads();
        if (threadIdx.x < 64) sRd[threadIdx.x] = threadIdx.x < w ? 1.0 / sL[threadIdx.x * (kLdsLd + 1)] : 0.0;
        if (nb > 0) load_chunk(Lb, ld, w + nb, w, w, true, pre);     // prefetch first below chunk
        __syncthreads();

        v4d xr[4];
        if (act) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * t + 4 * r + g;
                    const int row = row0 + i;
                    xr[t][r] = (i < w && row >= kstart) ? Xs[(int64_t)(row - kstart) * kTile + col] : 0.0;
                }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (16 * t < w) {
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        if (16 * t + k < w) {
                            const int gk = k & 3;
                            const int rk = k >> 2;
                            const double xk_own = xr[t][rk] * sRd[16 * t + k];
                            if (g == gk) xr[t][rk] = xk_own;
                            const double xk = __shfl(xk_own, j + 16 * gk, 64);
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int ii = 4 * r + g;
                                const double lik = sL[(16 * t + k) * kLdsLd + 16 * t + ii];
                                if (ii > k) xr[t][r] -= lik * xk;
                            }
                        }
                    }
#pragma unroll
                    for (int t2 = t + 1; t2 < 4; ++t2) {
                        if (16 * t2 < w) {
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                const double a = -sL[(16 * t + 4 * s + g) * kLdsLd + 16 * t2 + j];
                                xr[t2] = mfma_f64(a, xr[t][s], xr[t2]);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * t + 4 * r + g;
                    const int row = row0 + i;
                    if (i < w && row >= kstart) Xs[(int64_t)(row - kstart) * kTile + col] = xr[t][r];
                }
        }

        // ---- pruned rows below the block, 64 at a time
        const int32_t* __restrict__ rw = R + bd.rows_off;
        for (int q0 = 0; q0 < nb; q0 += 64) {
            __syncthreads();             // sL free (diagonal block or previous chunk)
            store_chunk(sL, pre);
            if (q0 + 64 < nb) load_chunk(Lb, ld, w + nb, w, w + q0 + 64, true, pre);
            __syncthreads();
            if (!act) continue;
            v4d acc[4];
            int32_t off[4][4];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q = q0 + 16 * rt + 4 * r + g;
                    off[rt][r] = q < nb ? (rw[q] - kstart) * kTile + col : -1;
                    acc[rt][r] = off[rt][r] >= 0 ? Xs[off[rt][r]] : 0.0;
                }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (16 * t < w) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const double* sk = sL + (16 * t + 4 * s + g) * kLdsLd + j;
#pragma unroll
                        for (int rt = 0; rt < 4; ++rt)
                            acc[rt] = mfma_f64(sk[16 * rt], xr[t][s], acc[rt]);
                    }
                }
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (off[rt][r] >= 0) Xs[off[rt][r]] = acc[rt][r];
        }
    }
}

// ---------------------------------------------------------------------------
// Staircase SYRK, F = X^T X (Sec. 3.3, output splitting): one workgroup per
// lower 64 x 64 tile (I >= J) of the sorted F; its k-range starts at the first
// pivot of tile I, which bounds the nonzero rows of both operands.  The
// result is written straight to the original multiplier order,
// F[pi(a), pi(b)] = F[pi(b), pi(a)] = sum_k X[k, a] X[k, b].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void syrk_stair_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const SyrkItem* __restrict__ items, const double* __restrict__ X,
    const int32_t* __restrict__ pi, double* __restrict__ F)
{
    constexpr int KC = 16;
    constexpr int LDP = kTile + 2;
    __shared__ double sI[KC * LDP];
    __shared__ double sJ[KC * LDP];
    const SyrkItem it = items[blockIdx.x];
    const SubDev S = subs[it.sub];
    const TileDev TI = tiles[S.tile_off + it.I];
    const TileDev TJ = tiles[S.tile_off + it.J];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const int wi = wv >> 1;
    const int wj = wv & 1;
    const bool diag = it.I == it.J;
    const bool active = !(diag && wi < wj);
    const int n = S.n;
    const double* __restrict__ XI = X + TI.x_off;
    const double* __restrict__ XJ = X + TJ.x_off;

    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

    for (int kb = TI.kstart; kb < n; kb += KC) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx >> 6;
            const int cc = idx & 63;
            const int k = kb + rr;
            sI[rr * LDP + cc] = k < n ? XI[(int64_t)(k - TI.kstart) * kTile + cc] : 0.0;
            sJ[rr * LDP + cc] = k < n ? XJ[(int64_t)(k - TJ.kstart) * kTile + cc] : 0.0;
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int s = 0; s < KC / 4; ++s) {
                const int kr = (4 * s + g) * LDP;
                const double a0 = sI[kr + 32 * wi + j];
                const double a1 = sI[kr + 32 * wi + 16 + j];
                const double b0 = sJ[kr + 32 * wj + j];
                const double b1 = sJ[kr + 32 * wj + 16 + j];
                acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
                acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
                acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
                acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
            }
        }
        __syncthreads();
    }
    if (!active) return;
    const int m = S.m;
    const int32_t* __restrict__ pis = pi + S.col_off;
    double* __restrict__ Fs = F + S.F_off;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = it.I * kTile + 32 * wi + 16 * ti + 4 * r + g;
                const int b = it.J * kTile + 32 * wj + 16 * tj + j;
                if (a < m && b < m && (!diag || a >= b)) {
                    const int64_t pa = pis[a];
                    const int64_t pb = pis[b];
                    const double v = acc[ti][tj][r];
                    Fs[pa + pb * m] = v;
                    Fs[pb + pa * m] = v;
                }
            }
}

// ---------------------------------------------------------------------------
hipError_t launch_assemble_f64(const DevTables& t, hipStream_t stream, hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    if (t.ntiles > 0)
        hipLaunchKernelGGL(trsm_stair_f64, dim3((unsigned)t.ntiles), dim3(256), 0, stream, t.subs,
                           t.tiles, t.blocks, t.rows, t.lval, t.piv, t.sgn, t.X);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], stream)) != hipSuccess) return e;
    if (t.nsyrk > 0)
        hipLaunchKernelGGL(syrk_stair_f64, dim3((unsigned)t.nsyrk), dim3(256), 0, stream, t.subs,
                           t.tiles, t.syrk, t.X, t.pi, t.F);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], stream)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace scasm
