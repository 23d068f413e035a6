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
// One workgroup = one 64-column tile of one subdomain; each wavefront owns a
// 16-column stripe and sweeps the factor blocks from the block holding the
// stripe's first pivot (rows above it are zero and stay zero: forward
// substitution only propagates downwards).  Per block:
//   1. the block's w (<= 64) rows of the stripe are loaded into registers;
//   2. diagonal solve in FP64: 16-row sub-blocks by substitution (division by
//      the diagonal, column-wise elimination), each followed by an MFMA
//      update of the sub-blocks below it inside the diagonal block;
//   3. the solved rows are stored and the pruned rows below the block are
//      updated, X[R_b] -= L[R_b, b] X[b], with FP64 MFMA, 16 rows at a time.
// The stripes never interact (columns of X are independent), so there is no
// workgroup barrier after initialisation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trsm_stair_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows,
    const double* __restrict__ lval, const int32_t* __restrict__ piv,
    const int8_t* __restrict__ sgn, double* __restrict__ X)
{
    __shared__ double ldiag[4][16 * 17];
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
    __threadfence_block();
    if (wv * kStripe >= T.ncols) return;

    const BlockDev* __restrict__ B = blocks + S.blk_off;
    const int32_t* __restrict__ R = rows + S.rows_off;
    const double* __restrict__ L = lval + S.lval_off;
    double* __restrict__ ld_s = ldiag[wv];

    for (int b = T.start_block[wv]; b < S.nblocks; ++b) {
        const BlockDev bd = B[b];
        const int w = bd.w;
        const int ld = bd.ld;
        const int row0 = bd.row0;
        const double* __restrict__ Lb = L + bd.lval_off;

        v4d xr[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * t + 4 * r + g;
                const int row = row0 + i;
                xr[t][r] = (i < w && row >= kstart) ? Xs[(int64_t)(row - kstart) * kTile + col] : 0.0;
            }

        // ---- diagonal block
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (16 * t < w) {
            wave_sync();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ii = 4 * r + g;
                double v = 0.0;
                if (16 * t + ii < w && 16 * t + j < w)
                    v = Lb[(int64_t)(16 * t + j) * ld + 16 * t + ii];
                ld_s[ii * 17 + j] = v;
            }
            wave_sync();
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (16 * t + k < w) {
                const int gk = k & 3;
                const int rk = k >> 2;
                const double xk_own = xr[t][rk] / ld_s[k * 17 + k];
                if (g == gk) xr[t][rk] = xk_own;
                const double xk = __shfl(xk_own, j + 16 * gk, 64);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ii = 4 * r + g;
                    const double lik = ld_s[ii * 17 + k];
                    if (ii > k) xr[t][r] -= lik * xk;
                }
                }
            }
#pragma unroll
            for (int t2 = t + 1; t2 < 4; ++t2) {
                if (16 * t2 < w) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int kc = 16 * t + 4 * s + g;
                    const int ir = 16 * t2 + j;
                    const double a = (kc < w && ir < w) ? -Lb[(int64_t)kc * ld + ir] : 0.0;
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

        // ---- pruned rows below the block
        const int nb = bd.nbelow;
        const int32_t* __restrict__ rw = R + bd.rows_off;
        const double* __restrict__ Lq = Lb + w;      // element (q, k) at Lq[k * ld + q]
        for (int q0 = 0; q0 < nb; q0 += 32) {
            v4d acc0, acc1;
            int64_t off0[4], off1[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int qa = q0 + 4 * r + g;
                const int qb = qa + 16;
                off0[r] = qa < nb ? (int64_t)(rw[qa] - kstart) * kTile + col : -1;
                off1[r] = qb < nb ? (int64_t)(rw[qb] - kstart) * kTile + col : -1;
                acc0[r] = off0[r] >= 0 ? Xs[off0[r]] : 0.0;
                acc1[r] = off1[r] >= 0 ? Xs[off1[r]] : 0.0;
            }
            const int qa = q0 + j;
            const int qb = qa + 16;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (16 * t < w) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int kc = 16 * t + 4 * s + g;
                    const bool kok = kc < w;
                    const double a0 = (kok && qa < nb) ? -Lq[(int64_t)kc * ld + qa] : 0.0;
                    const double a1 = (kok && qb < nb) ? -Lq[(int64_t)kc * ld + qb] : 0.0;
                    acc0 = mfma_f64(a0, xr[t][s], acc0);
                    acc1 = mfma_f64(a1, xr[t][s], acc1);
                }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (off0[r] >= 0) Xs[off0[r]] = acc0[r];
                if (off1[r] >= 0) Xs[off1[r]] = acc1[r];
            }
        }
        __threadfence_block();
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
hipError_t launch_assemble_f64(const DevTables& t, hipStream_t stream) {
    if (t.ntiles > 0)
        hipLaunchKernelGGL(trsm_stair_f64, dim3((unsigned)t.ntiles), dim3(256), 0, stream, t.subs,
                           t.tiles, t.blocks, t.rows, t.lval, t.piv, t.sgn, t.X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.nsyrk > 0)
        hipLaunchKernelGGL(syrk_stair_f64, dim3((unsigned)t.nsyrk), dim3(256), 0, stream, t.subs,
                           t.tiles, t.syrk, t.X, t.pi, t.F);
    return hipGetLastError();
}

}  // namespace scasm
