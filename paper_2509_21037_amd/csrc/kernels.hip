// HIP kernels for gfx950 (CDNA4, wave64): staircase TRSM and SYRK of the
// dual Schur-complement assembly (paper, Sec. 3.2 and 3.3), FP64 and mixed
// precision.  The solution-stage kernels are in apply.hip.
//
// MFMA operand layouts used throughout (v_mfma_f64_16x16x4f64):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   C/D (16x16): lane l, register r holds D[4 r + l / 16][l % 16]
// so the D registers of a 16 x 16 tile are, register r, exactly the B operand
// of k-slice r of the same tile used as a right-hand side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <type_traits>

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

typedef float v4f __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x4f32 takes A and B in the same lane layout as the FP64
// instruction, but its accumulator is laid out differently:
//   C/D (16x16): lane l, register r holds D[4 (l / 16) + r][l % 16].
__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Staircase TRSM, X = L^{-1} P B^T (Sec. 3.2, factor splitting with pruning).
// One workgroup = one 64-column tile of one subdomain; wavefront v owns the
// 16-column stripe v and holds the X rows of the current factor block in
// registers (FP64 accumulator layout).  The four wavefronts walk the factor
// blocks together, from the block holding the tile's first pivot (rows above
// it are zero and stay zero: forward substitution only propagates
// downwards); a stripe whose first pivot lies further down joins at its own
// first block.  Per block b:
//   1. X[b] <- L_bb^{-1} X[b], FP64 MFMA with the inverse of the diagonal
//      block computed on the host (its lower 16 x 4 tiles, one chunk);
//   2. the pruned rows below the block, 32 at a time (64 in mixed precision):
//      X[R_b] -= L[R_b, b] X[b] (MFMA, rows gathered and scattered).
// The factor flows through the workgroup as a stream of chunks (the inverse
// of a diagonal block, up to 20 KB, or 16 KB of pruned-row tiles): while
// chunk c is used from LDS, chunks c+1 and c+2 are in registers (loaded two
// steps ahead: one step of latency hiding was measured 23% slower); c+1 is
// written to the other half of a double buffer at the end of the step; one
// barrier per chunk, on LDS only (X columns of a stripe are private to its
// wavefront, so no barrier waits on global memory).  Rows of the next chunk
// of the same block are gathered before the current chunk's MFMAs (the
// chunks of one block update disjoint rows); a wavefront reads rows it wrote
// itself in program order.
// Mixed precision: the same with FP32 X and FP32 A tiles / MFMA for step 2;
// step 1 stays FP64 (the block rows are widened, solved, rounded back).
// Merged pairs: two consecutive blocks b, b + 1 that a tile visits one after
// the other and whose rows below nest, R_b = rows(b + 1) followed by R_{b+1}
// (BlockDev::flags, set by the host: two panels of one supernode, or a child
// block with its parent's structure).  Block b then
// updates only the rows of b + 1; its solved rows -X[b] wait in LDS (one 64 x
// 16 slot per wavefront); block b + 1 updates R_{b+1} once with both:
// X[R] -= L[R, b] X[b] + L[R, b + 1] X[b + 1], two chunk steps per row group
// (the A tiles of b, then those of b + 1), one gather and one scatter.  The
// sums run in the same order as two separate updates (a read-modify-write in
// the X precision is exact), so X and F are bit for bit the same; the rows
// below are read and written once instead of twice.
// ---------------------------------------------------------------------------
// a chunk: the 40 lower tiles of a 64 x 64 diagonal inverse (20 KB), or 16 KB
// of pruned-row tiles
constexpr int kChunkBytes = 40 * 64 * 8;
constexpr int kIdxBytes = 64 * 4;                // row indices carried by a chunk (up to 64)
constexpr int kBufBytes = kChunkBytes + kIdxBytes;
constexpr int kTrsmSmem = 2 * kBufBytes;

// Barrier that waits for this wavefront's LDS traffic only: global loads in
// flight (prefetches, gathers) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

struct ChunkSrc {
    const char* p;       // always a valid address (the subdomain's factor when bytes == 0)
    int bytes;
    bool has_idx;        // the chunk carries the row indices at ip
    const int32_t* ip;   // row indices of the pruned chunk gathered next (64 are read);
                         // always a valid address (the row array is padded by 64 entries)
};

// Register prefetch of one chunk: five 16-byte pieces per thread, loaded
// unconditionally (pieces past the chunk re-read its first bytes), plus the
// 32 row indices (threads 0..7 keep them).  Separate registers, not a struct:
// the prefetch must stay out of scratch memory.
__device__ __forceinline__ void chunk_load(uint4& v0, uint4& v1, uint4& v2, uint4& v3, uint4& v4, uint4& vi,
                                           const ChunkSrc& s) {
    const int e = threadIdx.x * 16;
    v0 = *reinterpret_cast<const uint4*>(s.p + (e < s.bytes ? e : 0));
    v1 = *reinterpret_cast<const uint4*>(s.p + (e + 4096 < s.bytes ? e + 4096 : 0));
    v2 = *reinterpret_cast<const uint4*>(s.p + (e + 8192 < s.bytes ? e + 8192 : 0));
    v3 = *reinterpret_cast<const uint4*>(s.p + (e + 12288 < s.bytes ? e + 12288 : 0));
    v4 = *reinterpret_cast<const uint4*>(s.p + (e + 16384 < s.bytes ? e + 16384 : 0));
    vi = *reinterpret_cast<const uint4*>(s.ip + 4 * (threadIdx.x & 15));
}

__device__ __forceinline__ void chunk_store(const uint4& v0, const uint4& v1, const uint4& v2, const uint4& v3,
                                            const uint4& v4, const uint4& vi, char* __restrict__ dst,
                                            const ChunkSrc& s) {
    const int e = threadIdx.x * 16;
    if (e < s.bytes) *reinterpret_cast<uint4*>(dst + e) = v0;
    if (e + 4096 < s.bytes) *reinterpret_cast<uint4*>(dst + e + 4096) = v1;
    if (e + 8192 < s.bytes) *reinterpret_cast<uint4*>(dst + e + 8192) = v2;
    if (e + 12288 < s.bytes) *reinterpret_cast<uint4*>(dst + e + 12288) = v3;
    if (e + 16384 < s.bytes) *reinterpret_cast<uint4*>(dst + e + 16384) = v4;
    if (s.has_idx && threadIdx.x < 16) *reinterpret_cast<uint4*>(dst + kChunkBytes + 16 * threadIdx.x) = vi;
}

// Scalar copy of the block descriptor fields the TRSM uses.
struct BlockLite {
    int w, nb;
    int64_t aoff, linv_off, rows_off;
};

__device__ __forceinline__ BlockLite block_lite(const BlockDev* __restrict__ B, int b) {
    return {B[b].w, B[b].nbelow, B[b].aoff, B[b].linv_off, B[b].rows_off};
}

// Pruned row tiles per chunk: 16 KB of A tiles, two FP64 or four FP32 row
// tiles of 16 k-slices.
template <class TA>
constexpr int kPruneTiles = sizeof(TA) == 8 ? 2 : 4;

// Role of a visit in a merged pair (see above): 0 = alone, 1 = first block
// (updates only the rows of the next block), 2 = second block (its update of
// the rows below also applies the first block's).
__device__ __forceinline__ int visit_role(const BlockDev* __restrict__ B, const int32_t* __restrict__ V, int k,
                                          int nv, int prev_role) {
    if (prev_role == 1) return 2;
    return (k + 1 < nv && B[V[k]].flags != 0 && V[k + 1] == V[k] + 1) ? 1 : 0;
}

// Rows the update of a visit covers: the rows of the next block (role 1,
// whole 16-row tiles), else the block's pruned rows.
__device__ __forceinline__ int update_rows(const BlockDev* __restrict__ B, const int32_t* __restrict__ V, int k,
                                           int role, int nb) {
    return role == 1 ? B[V[k] + 1].w : nb;
}

// Chunk c of a visit (block bd, role, `urows` rows in its update; prev = the
// first block of the pair for role 2): c = 0 is the inverse of the diagonal
// block (its lower tiles), the rest groups of kPruneTiles pruned row tiles
// (TA = precision of the update's A tiles); role 2 alternates the first
// block's A tiles of a row group (its pruned rows from the second block's
// width on) with the second block's.  The diagonal chunk carries the row
// indices of the first row group, the (second) chunk of row group p those of
// group p + 1: they are gathered while the chunk is in use.
template <class TA>
__device__ __forceinline__ ChunkSrc chunk_src(const BlockLite& bd, int prev_w, int64_t prev_aoff, int role, int urows,
                                              int c, const double* __restrict__ L, const TA* __restrict__ LA,
                                              const int32_t* __restrict__ R) {
    const int nks = (bd.w + 3) >> 2;
    const int nrt_d = (bd.w + 15) >> 4;
    constexpr int PT = kPruneTiles<TA>;
    const int nrt = (urows + 15) >> 4;
    const int np = (nrt + PT - 1) / PT;
    if (c == 0)
        return {reinterpret_cast<const char*>(L + bd.linv_off), (2 * (nrt_d - 1) * nrt_d + nks) * 64 * 8, np > 0,
                R + bd.rows_off};
    const int p = role == 2 ? (c - 1) >> 1 : c - 1;
    const int nt = min(PT, nrt - PT * p);
    if (role == 2 && ((c - 1) & 1) == 0) {
        const int nks1 = (prev_w + 3) >> 2;
        return {reinterpret_cast<const char*>(LA + prev_aoff + (int64_t)((bd.w >> 4) + PT * p) * nks1 * 64),
                nt * nks1 * 64 * (int)sizeof(TA), false, R};
    }
    return {reinterpret_cast<const char*>(LA + bd.aoff + (int64_t)PT * p * nks * 64),
            nt * nks * 64 * (int)sizeof(TA), p + 1 < np, R + bd.rows_off + 16 * PT * min(p + 1, np - 1)};
}

// LDS slot of the first block's solved rows: 16 values per lane and wavefront.
template <class TX>
constexpr int kSlotBytes = 4 * 16 * 64 * (int)sizeof(TX);

template <bool MIXED, bool MERGE>
__device__ __forceinline__ void trsm_tile(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ visit, const uint64_t* __restrict__ vrows,
    const double* __restrict__ lval, const float* __restrict__ lval32,
    const int32_t* __restrict__ piv, const int8_t* __restrict__ sgn,
    typename std::conditional<MIXED, float, double>::type* __restrict__ X, int ti, char* __restrict__ smem)
{
    using TX = typename std::conditional<MIXED, float, double>::type;
    using VX = typename std::conditional<MIXED, v4f, v4d>::type;
    constexpr int PT = kPruneTiles<TX>;          // pruned row tiles per chunk
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const TileDev T = tiles[ti];
    const SubDev S = subs[T.sub];
    const int kstart = T.kstart;
    TX* __restrict__ Xs = X + T.x_off;
    const int col = wv * kStripe + j;
    const int64_t cbase = S.col_off + (int64_t)T.tile * kTile;
    const BlockDev* __restrict__ B = blocks + S.blk_off;
    const int32_t* __restrict__ R = rows + S.rows_off;
    const double* __restrict__ L = lval + S.lval_off;
    const TX* __restrict__ LA;
    if constexpr (MIXED) LA = lval32 + S.lval_off;
    else LA = lval + S.lval_off;
    const int my_start = tiles[ti].start_block[wv];
    // the blocks this tile visits, increasing: those holding rows on the
    // elimination-tree paths of its pivots (all other rows of X are zero)
    const int nv = T.nvisit;
    const int32_t* __restrict__ V = visit + T.visit_off;
    // per visit, the rows of the block on the paths: the others are zero
    // before and after its diagonal solve and are neither read nor written
    const uint64_t* __restrict__ VR = vrows + T.visit_off;

    // right-hand side P B^T: sign at the pivot row, zero elsewhere.  Only the
    // 16-row steps of visited blocks that hold a row on the paths are cleared:
    // the other rows are off every path, the sweep writes them at most with
    // exact-zero updates of whatever they held, the diagonal step neither
    // reads nor writes them, and the SYRK reads only the steps of a slab that
    // hold a row on its paths
    for (int k = 0; k < nv; ++k) {
        const int r0 = B[V[k]].row0;
        const int r1 = r0 + B[V[k]].w;
        const uint64_t on = VR[k];
        for (int q = 0; q < 4; ++q) {
            if (((on >> (16 * q)) & 0xFFFFull) == 0) continue;
            const int qe = min(r0 + 16 * (q + 1), r1);
            for (int r = max(r0 + 16 * q, kstart) + g; r < qe; r += 4) Xs[(int64_t)(r - kstart) * kTile + col] = TX(0);
        }
    }
    __threadfence_block();
    if (g == 0 && col < T.ncols) Xs[(int64_t)(piv[cbase + col] - kstart) * kTile + col] = (TX)sgn[cbase + col];
    if (nv <= 0) return;

    BlockLite bd = block_lite(B, V[0]);
    TX* __restrict__ slot = reinterpret_cast<TX*>(smem + kTrsmSmem) + wv * 16 * 64;
    // prefetch cursor over the flattened chunk stream: chunk s+2 is loaded
    // into registers at the start of step s, chunk s+1 goes to LDS at its end
    int pk = 0, pc = 0;
    BlockLite pbd = bd;
    int pprev_w = 0;
    int64_t pprev_aoff = 0;
    int prole = MERGE ? visit_role(B, V, 0, nv, 0) : 0;
    int purows = update_rows(B, V, 0, prole, pbd.nb);
    auto nchunks = [](int role, int urows) {
        const int np = (((urows + 15) >> 4) + PT - 1) / PT;
        return 1 + (role == 2 ? 2 * np : np);
    };
    int pnch = nchunks(prole, purows);
    auto take = [&]() {
        ChunkSrc c{reinterpret_cast<const char*>(L), 0, false, R};
        if (pk < nv) {
            c = chunk_src(pbd, pprev_w, pprev_aoff, prole, purows, pc, L, LA, R);
            if (++pc >= pnch) {
                ++pk;
                pc = 0;
                if (pk < nv) {
                    pprev_w = pbd.w;
                    pprev_aoff = pbd.aoff;
                    pbd = block_lite(B, V[pk]);
                    prole = MERGE ? visit_role(B, V, pk, nv, prole) : 0;
                    purows = update_rows(B, V, pk, prole, pbd.nb);
                    pnch = nchunks(prole, purows);
                }
            }
        }
        return c;
    };
    // a*: chunk s+1 (stored to LDS at the end of step s), b*: chunk s+2;
    // sa_* / sb_* describe them
    uint4 a0, a1, a2, a3, a4, ai, b0, b1, b2, b3, b4, bi;
    {
        const ChunkSrc c0 = take();
        chunk_load(a0, a1, a2, a3, a4, ai, c0);
        chunk_store(a0, a1, a2, a3, a4, ai, smem, c0);
    }
    const char* sa_p; int sa_bytes; bool sa_idx; const int32_t* sa_ip;
    const char* sb_p = reinterpret_cast<const char*>(L); int sb_bytes = 0; bool sb_idx = false; const int32_t* sb_ip = R;
    {
        const ChunkSrc c1 = take();
        chunk_load(a0, a1, a2, a3, a4, ai, c1);
        sa_p = c1.p; sa_bytes = c1.bytes; sa_idx = c1.has_idx; sa_ip = c1.ip;
    }
    lds_barrier();
    int buf = 0;

    auto step_begin = [&]() {
        const ChunkSrc cb = take();
        chunk_load(b0, b1, b2, b3, b4, bi, cb);
        sb_p = cb.p; sb_bytes = cb.bytes; sb_idx = cb.has_idx; sb_ip = cb.ip;
    };
    auto step_end = [&]() {
        if (sa_bytes > 0) {
            const ChunkSrc ca{sa_p, sa_bytes, sa_idx, sa_ip};
            chunk_store(a0, a1, a2, a3, a4, ai, smem + (buf ^ 1) * kBufBytes, ca);
            lds_barrier();
            buf ^= 1;
        }
        a0 = b0; a1 = b1; a2 = b2; a3 = b3; a4 = b4; ai = bi;
        sa_p = sb_p; sa_bytes = sb_bytes; sa_idx = sb_idx; sa_ip = sb_ip;
    };
    int role = 0;
    int nks_prev = 0;                            // k-slices of the pair's first block (role 2)
    for (int k = 0; k < nv; ++k) {
        const int b = V[k];
        const uint64_t on = VR[k] >> g;          // bit 16t + 4r: row 16t + 4r + g of the block
        const int w = bd.w;
        const int row0 = B[b].row0;
        role = MERGE ? visit_role(B, V, k, nv, role) : 0;
        const int nb = update_rows(B, V, k, role, bd.nb);   // rows this visit's update covers
        const int nks = (w + 3) >> 2;
        const int nrt_d = (w + 15) >> 4;
        const int nrt = (nb + 15) >> 4;
        const int np = (nrt + PT - 1) / PT;
        const bool act = b >= my_start;
        const BlockLite bn = block_lite(B, V[k + 1 < nv ? k + 1 : k]);

        VX accn[PT];                             // rows of the next pruned chunk
        int offn[PT][4];
        auto gather = [&](int p) {               // row indices from the chunk in LDS
            const int32_t* __restrict__ sidx = reinterpret_cast<const int32_t*>(smem + buf * kBufBytes + kChunkBytes);
#pragma unroll
            for (int u = 0; u < PT; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * u + (MIXED ? 4 * g + r : 4 * r + g);
                    offn[u][r] = 16 * PT * p + k < nb ? (sidx[k] - kstart) * kTile + col : -1;
                    accn[u][r] = offn[u][r] >= 0 ? Xs[offn[u][r]] : TX(0);
                }
        };

        // ---- 1. X[b] <- L_bb^{-1} X[b]
        TX xb[4][4];                             // -X[b]: B operands of step 2
        {
            v4d xr[4];
            if (act) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * t + 4 * r + g;
                        const int row = row0 + i;
                        xr[t][r] = (((on >> (16 * t + 4 * r)) & 1) && row >= kstart)
                                       ? (double)Xs[(int64_t)(row - kstart) * kTile + col] : 0.0;
                    }
                if (np > 0) gather(0);
            }
            step_begin();
            if (act) {
                // lower tiles only: row tile u needs k-slices of row tiles t <= u
                const double* __restrict__ sA = reinterpret_cast<const double*>(smem + buf * kBufBytes);
                v4d tmp[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    tmp[u] = v4d{0.0, 0.0, 0.0, 0.0};
                    if (u < nrt_d) {
#pragma unroll
                        for (int t = 0; t <= u; ++t)
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                const int ks = 4 * t + s;
                                if (ks < nks) tmp[u] = mfma_f64(sA[(2 * u * (u + 1) + ks) * 64 + lane], xr[t][s], tmp[u]);
                            }
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (u < nrt_d) xr[u] = tmp[u];
            }
            step_end();
            if (act) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * t + 4 * r + g;
                        const int row = row0 + i;
                        const TX v = (TX)xr[t][r];
                        if (((on >> (16 * t + 4 * r)) & 1) && row >= kstart)
                            Xs[(int64_t)(row - kstart) * kTile + col] = v;
                        xb[t][r] = -v;
                    }
            }
            // the first block of a pair keeps its solved rows for the second
            // (zero for a wavefront that starts at the second)
            if (role == 1) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) slot[(4 * t + r) * 64 + lane] = act ? xb[t][r] : TX(0);
            }
        }

        // ---- 2. X[R_b] -= L[R_b, b] X[b], pruned row tiles PT p .. PT p + PT - 1
        // (role 2: first the pair's first block's A tiles with its solved
        // rows from LDS, then this block's, one gather and one scatter)
        VX acc[PT];
        int off[PT][4];
        for (int p = 0; p < np; ++p) {
            if (role == 2) {
                if constexpr (MIXED) step_begin();
                if (act) {
#pragma unroll
                    for (int u = 0; u < PT; ++u) {
                        acc[u] = accn[u];
#pragma unroll
                        for (int r = 0; r < 4; ++r) off[u][r] = offn[u][r];
                    }
                }
                if constexpr (!MIXED) step_begin();
                if (act) {
                    const TX* __restrict__ sA = reinterpret_cast<const TX*>(smem + buf * kBufBytes);
                    const int nt = min(PT, nrt - PT * p);
#pragma unroll
                    for (int u = 0; u < PT; ++u) {
                        if (u < nt) {
#pragma unroll
                            for (int t = 0; t < 4; ++t)
#pragma unroll
                                for (int s = 0; s < 4; ++s) {
                                    const int ks = 4 * t + s;
                                    if (ks < nks_prev) {
                                        const TX xv = slot[ks * 64 + lane];
                                        if constexpr (MIXED) acc[u] = mfma_f32(sA[(u * nks_prev + ks) * 64 + lane], xv, acc[u]);
                                        else acc[u] = mfma_f64(sA[(u * nks_prev + ks) * 64 + lane], xv, acc[u]);
                                    }
                                }
                        }
                    }
                }
                step_end();
            }
            // FP64: the next gather is issued before the next chunk's loads, so
            // that waiting for it a step later does not wait for them as well
            // (the mixed kernel has no registers left for that order)
            if constexpr (MIXED) step_begin();
            if (act) {
                if (role != 2) {
#pragma unroll
                    for (int u = 0; u < PT; ++u) {
                        acc[u] = accn[u];
#pragma unroll
                        for (int r = 0; r < 4; ++r) off[u][r] = offn[u][r];
                    }
                }
                if (p + 1 < np) gather(p + 1);
            }
            if constexpr (!MIXED) step_begin();
            if (act) {
                const TX* __restrict__ sA = reinterpret_cast<const TX*>(smem + buf * kBufBytes);
                const int nt = min(PT, nrt - PT * p);
#pragma unroll
                for (int u = 0; u < PT; ++u) {
                    if (u < nt) {
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                const int ks = 4 * t + s;
                                if (ks < nks) {
                                    if constexpr (MIXED) acc[u] = mfma_f32(sA[(u * nks + ks) * 64 + lane], xb[t][s], acc[u]);
                                    else acc[u] = mfma_f64(sA[(u * nks + ks) * 64 + lane], xb[t][s], acc[u]);
                                }
                            }
                    }
                }
#pragma unroll
                for (int u = 0; u < PT; ++u)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (off[u][r] >= 0) Xs[off[u][r]] = acc[u][r];
            }
            step_end();
        }
        nks_prev = nks;
        bd = bn;
    }
}

// MERGE: with the merged pairs (BlockDev::flags); without, the flags are
// ignored and the merged code paths compile away.
template <bool MERGE>
__global__ __launch_bounds__(256, 2) void trsm_stair_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows, const int32_t* __restrict__ visit,
    const uint64_t* __restrict__ vrows, const double* __restrict__ lval, const int32_t* __restrict__ piv,
    const int8_t* __restrict__ sgn, const int32_t* __restrict__ order, double* __restrict__ X)
{
    __shared__ __align__(16) char smem[kTrsmSmem + (MERGE ? kSlotBytes<double> : 0)];
    const int ti = order[blockIdx.x];
    if (ti < 0) return;
    trsm_tile<false, MERGE>(subs, tiles, blocks, rows, visit, vrows, lval, nullptr, piv, sgn, X, ti, smem);
}

template <bool MERGE>
__global__ __launch_bounds__(256, 2) void trsm_stair_mixed(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows, const int32_t* __restrict__ visit,
    const uint64_t* __restrict__ vrows, const double* __restrict__ lval, const float* __restrict__ lval32,
    const int32_t* __restrict__ piv,
    const int8_t* __restrict__ sgn, const int32_t* __restrict__ order, float* __restrict__ X)
{
    __shared__ __align__(16) char smem[kTrsmSmem + (MERGE ? kSlotBytes<float> : 0)];
    const int ti = order[blockIdx.x];
    if (ti < 0) return;
    trsm_tile<true, MERGE>(subs, tiles, blocks, rows, visit, vrows, lval, lval32, piv, sgn, X, ti, smem);
}

// ---------------------------------------------------------------------------
// Staircase SYRK, F = X^T X (Sec. 3.3, output splitting): one workgroup per
// 64 x 64 block (I >= J, in units of 64-column X tiles) of the lower triangle
// of the column-sorted F; wavefront w computes its rows 16w .. 16w + 15
// (1 x 4 MFMA tiles).  The k-range is the block's list of 16-row steps: those
// where both X tiles hold rows on the elimination-tree paths of their pivots
// (every other step adds zero products; the staircase bound, rows below the
// first pivot of tile I, is the outer limit of that set).  Blocks with an
// empty list are structurally zero and are not launched: the plan clears F
// once when it is created.  Used for subdomains up to kSyrkBlockMaxN rows
// (FP32: kSyrkBlockMaxNMixed), whose X slabs largely stay in L2 while their
// blocks re-read them.  X rows are staged through double-buffered LDS, 16
// rows per step, the next step prefetched into registers.  F stays in the
// sorted column order (the permutation back to the multiplier order is
// applied to the vectors of the apply and by sc_get_F), stored as the lower
// triangle of 128 x 128 tiles, tile (I, J) at I(I+1)/2 + J, each row-major,
// diagonal tiles whole: block (2T+1, 2T) also writes its transpose, the upper
// quadrant of diagonal tile T.  Columns past m are never written and stay
// zero.
// ---------------------------------------------------------------------------
constexpr int kSyrkKC = 16;                  // X rows per step
constexpr int kSyrkLd = kTile + 4;           // LDS row stride (elements)

template <class TX>
constexpr int kSyrkSmem = 4 * kSyrkKC * kSyrkLd * (int)sizeof(TX);

template <bool MIXED>
__device__ __forceinline__ void syrk_block(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles, const SyrkItem it,
    const int32_t* __restrict__ ksteps, const typename std::conditional<MIXED, float, double>::type* __restrict__ X,
    typename std::conditional<MIXED, float, double>::type* __restrict__ F, char* __restrict__ smem)
{
    using TX = typename std::conditional<MIXED, float, double>::type;
    using VX = typename std::conditional<MIXED, v4f, v4d>::type;
    using LV = typename std::conditional<MIXED, float4, double2>::type;
    constexpr int kVec = sizeof(LV) / sizeof(TX);                // elements per load
    constexpr int kPer = kSyrkKC * kTile / kVec / 256;           // loads per thread and slab
    TX (*sA)[kSyrkKC * kSyrkLd] = reinterpret_cast<TX (*)[kSyrkKC * kSyrkLd]>(smem);
    TX (*sB)[kSyrkKC * kSyrkLd] = sA + 2;
    const SubDev S = subs[it.sub];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const int n = S.n;
    const bool diag = it.I == it.J;          // one slab: sB aliases sA
    const TileDev& TI = tiles[S.tile_off + it.I];
    const TileDev& TJ = tiles[S.tile_off + it.J];
    const TX* __restrict__ xi = X + TI.x_off;
    const TX* __restrict__ xj = X + TJ.x_off;
    const int ki = TI.kstart, kj = TJ.kstart;
    const int32_t* __restrict__ KS = ksteps + it.step_off;
    const int nsteps = it.nsteps;

    VX acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = TX(0);

    LV rA[kPer], rB[kPer];
    auto load_step = [&](int kb) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx / (kTile / kVec);
            const int cc = kVec * (idx % (kTile / kVec));
            const int k = kb + rr;
            if (k < n && k >= ki) rA[e] = *reinterpret_cast<const LV*>(xi + (int64_t)(k - ki) * kTile + cc);
            else rA[e] = LV{};
            if (!diag && k < n && k >= kj) rB[e] = *reinterpret_cast<const LV*>(xj + (int64_t)(k - kj) * kTile + cc);
            else rB[e] = LV{};
        }
    };
    auto store_step = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx / (kTile / kVec);
            const int cc = kVec * (idx % (kTile / kVec));
            *reinterpret_cast<LV*>(&sA[buf][rr * kSyrkLd + cc]) = rA[e];
            if (!diag) *reinterpret_cast<LV*>(&sB[buf][rr * kSyrkLd + cc]) = rB[e];
        }
    };

    if (nsteps > 0) {
        load_step(KS[0]);
        store_step(0);
    }
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        const int buf = st & 1;
        if (st + 1 < nsteps) load_step(KS[st + 1]);
        const TX* __restrict__ pa = &sA[buf][g * kSyrkLd + 16 * wv + j];
        const TX* __restrict__ pb = &(diag ? sA : sB)[buf][g * kSyrkLd + j];
#pragma unroll
        for (int s = 0; s < kSyrkKC / 4; ++s) {
            const TX a = pa[4 * s * kSyrkLd];
            TX b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = pb[4 * s * kSyrkLd + 16 * t];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if constexpr (MIXED) acc[t] = mfma_f32(a, b[t], acc[t]);
                else acc[t] = mfma_f64(a, b[t], acc[t]);
            }
        }
        if (st + 1 < nsteps) store_step(buf ^ 1);
        __syncthreads();
    }
    const int I2 = it.I >> 1, J2 = it.J >> 1;
    TX* __restrict__ Ft = F + S.F_off + (int64_t)(I2 * (I2 + 1) / 2 + J2) * kFTileElems;
    const bool mirror = I2 == J2 && !diag;
    const int r0 = 64 * (it.I & 1) + 16 * wv;
    const int c0 = 64 * (it.J & 1);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + (MIXED ? 4 * g + r : 4 * r + g);
            const int col = c0 + 16 * t + j;
            Ft[row * kSyrkTile + col] = acc[t][r];
            if (mirror) Ft[col * kSyrkTile + row] = acc[t][r];
        }
}

__global__ __launch_bounds__(256) void syrk_block_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const SyrkItem* __restrict__ items, const int32_t* __restrict__ ksteps, const double* __restrict__ X,
    double* __restrict__ F)
{
    __shared__ __align__(16) char smem[kSyrkSmem<double>];
    const SyrkItem it = items[blockIdx.x];
    if (it.sub < 0) return;
    syrk_block<false>(subs, tiles, it, ksteps, X, F, smem);
}

// ---------------------------------------------------------------------------
// The same SYRK over 128 x 128 tiles (I >= J in units of kSyrkTile), each
// wavefront a 64 x 64 quadrant (4 x 4 MFMA tiles): twice the MFMA work per
// byte of X of the 64 x 64 blocks, used for the subdomains whose X slabs are
// too large to be re-read from L2 (n above kSyrkBlockMaxN, FP32 above
// kSyrkBlockMaxNMixed).  The k-range is the
// tile's list of 16-row steps where both column halves can hold nonzero rows;
// each entry marks which of the four 64-column slabs have nonzero rows in
// the step (bits at kStepSlabShift), the others read as zero (their rows may
// never have been written).  Diagonal tiles are computed whole.
// ---------------------------------------------------------------------------
constexpr int kWideLd = kSyrkTile + 4;
constexpr int kWideSmem = 4 * kSyrkKC * kWideLd * 8;

__device__ __forceinline__ void syrk_tile_item_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles, const SyrkItem it,
    const int32_t* __restrict__ ksteps, const double* __restrict__ X, double* __restrict__ F,
    char* __restrict__ smem)
{
    double (*sI)[kSyrkKC * kWideLd] = reinterpret_cast<double (*)[kSyrkKC * kWideLd]>(smem);
    double (*sJ)[kSyrkKC * kWideLd] = sI + 2;
    const SubDev S = subs[it.sub];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const int wi = wv >> 1;
    const int wj = wv & 1;
    const int n = S.n;

    // the two 64-column slabs of each 128-column tile (the second may not exist)
    const double* xs[4];
    int ks[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t64 = 2 * (q < 2 ? it.I : it.J) + (q & 1);
        if (t64 < S.ntiles) {
            const TileDev& T = tiles[S.tile_off + t64];
            xs[q] = X + T.x_off;
            ks[q] = T.kstart;
        } else {
            xs[q] = nullptr;
            ks[q] = INT_MAX;
        }
    }
    const int32_t* __restrict__ KS = ksteps + it.step_off;

    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};

    // thread -> (row, column pair) of a 16 x 128 step, 4 pairs per operand;
    // a slab whose bit is clear in the step entry holds no nonzero row there
    // (its rows may never have been written) and reads as zero
    double2 rI[4], rJ[4];
    auto load_step = [&](int ent) {
        const int kb = ent & kStepRowMask;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx >> 6;
            const int cc = 2 * (idx & 63);
            const int half = cc >> 6;
            const int c = cc & 63;
            const int k = kb + rr;
            const int qi = half, qj = 2 + half;
            const bool li = ((ent >> (kStepSlabShift + qi)) & 1) && k < n && k >= ks[qi];
            const bool lj = ((ent >> (kStepSlabShift + qj)) & 1) && k < n && k >= ks[qj];
            rI[e] = li ? *reinterpret_cast<const double2*>(xs[qi] + (int64_t)(k - ks[qi]) * kTile + c)
                       : make_double2(0.0, 0.0);
            rJ[e] = lj ? *reinterpret_cast<const double2*>(xs[qj] + (int64_t)(k - ks[qj]) * kTile + c)
                       : make_double2(0.0, 0.0);
        }
    };
    auto store_step = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx >> 6;
            const int cc = 2 * (idx & 63);
            *reinterpret_cast<double2*>(&sI[buf][rr * kWideLd + cc]) = rI[e];
            *reinterpret_cast<double2*>(&sJ[buf][rr * kWideLd + cc]) = rJ[e];
        }
    };

    const int nsteps = it.nsteps;
    if (nsteps > 0) {
        load_step(KS[0]);
        store_step(0);
    }
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        const int buf = st & 1;
        if (st + 1 < nsteps) load_step(KS[st + 1]);
        {
#pragma unroll
            for (int s = 0; s < kSyrkKC / 4; ++s) {
                const double* ai = &sI[buf][(4 * s + g) * kWideLd + 64 * wi + j];
                const double* bj = &sJ[buf][(4 * s + g) * kWideLd + 64 * wj + j];
                double a[4], b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    a[t] = ai[16 * t];
                    b[t] = bj[16 * t];
                }
#pragma unroll
                for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = mfma_f64(a[ti], b[tj], acc[ti][tj]);
            }
        }
        if (st + 1 < nsteps) store_step(buf ^ 1);
        __syncthreads();
    }
    double* __restrict__ Ft = F + S.F_off + (int64_t)(it.I * (it.I + 1) / 2 + it.J) * kFTileElems;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Ft[(64 * wi + 16 * ti + 4 * r + g) * kSyrkTile + 64 * wj + 16 * tj + j] = acc[ti][tj][r];
}

__global__ __launch_bounds__(256) void syrk_tile_f64(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const SyrkItem* __restrict__ items, const int32_t* __restrict__ ksteps, const double* __restrict__ X,
    double* __restrict__ F)
{
    __shared__ __align__(16) char smem[kWideSmem];
    const SyrkItem it = items[blockIdx.x];
    if (it.sub < 0) return;
    syrk_tile_item_f64(subs, tiles, it, ksteps, X, F, smem);
}

// ---------------------------------------------------------------------------
// Mixed precision (FP64 diagonal solves; FP32 X, off-diagonal updates and
// SYRK with FP32 MFMA and FP32 accumulation).
// ---------------------------------------------------------------------------

// FP64 factor values -> FP32 copy (round to nearest even).
__global__ __launch_bounds__(256) void convert_f64_f32(const double* __restrict__ a, float* __restrict__ b,
                                                       int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = (float)a[i];
}
// FP32 SYRK over 64 x 64 blocks: as syrk_block_f64 with FP32 X, FP32 MFMA and
// FP32 accumulation; F stored FP32.
__global__ __launch_bounds__(256) void syrk_block_f32(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const SyrkItem* __restrict__ items, const int32_t* __restrict__ ksteps, const float* __restrict__ X,
    float* __restrict__ F)
{
    __shared__ __align__(16) char smem[kSyrkSmem<float>];
    const SyrkItem it = items[blockIdx.x];
    if (it.sub < 0) return;
    syrk_block<true>(subs, tiles, it, ksteps, X, F, smem);
}

// FP32 SYRK over 128 x 128 tiles: as syrk_tile_f64 with FP32 X, FP32 MFMA and
// FP32 accumulation (33 KB of LDS: 4 workgroups per CU); F stored FP32.
constexpr int kWideSmemF = 4 * kSyrkKC * kWideLd * 4;

__device__ __forceinline__ void syrk_tile_item_f32(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles, const SyrkItem it,
    const int32_t* __restrict__ ksteps, const float* __restrict__ X, float* __restrict__ F,
    char* __restrict__ smem)
{
    float (*sI)[kSyrkKC * kWideLd] = reinterpret_cast<float (*)[kSyrkKC * kWideLd]>(smem);
    float (*sJ)[kSyrkKC * kWideLd] = sI + 2;
    const SubDev S = subs[it.sub];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int j = lane & 15;
    const int wi = wv >> 1;
    const int wj = wv & 1;
    const int n = S.n;

    const float* xs[4];
    int ks[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t64 = 2 * (q < 2 ? it.I : it.J) + (q & 1);
        if (t64 < S.ntiles) {
            const TileDev& T = tiles[S.tile_off + t64];
            xs[q] = X + T.x_off;
            ks[q] = T.kstart;
        } else {
            xs[q] = nullptr;
            ks[q] = INT_MAX;
        }
    }
    const int32_t* __restrict__ KS = ksteps + it.step_off;
    // a diagonal tile reads one slab pair (sJ aliases sI)
    const bool diag = it.I == it.J;

    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};

    // thread -> (row, 4 columns) of a 16 x 128 step, 2 per operand
    float4 rI[kSyrkKC / 8], rJ[kSyrkKC / 8];
    auto load_step = [&](int ent) {
        const int kb = ent & kStepRowMask;
#pragma unroll
        for (int e = 0; e < kSyrkKC / 8; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx >> 5;
            const int cc = 4 * (idx & 31);
            const int half = cc >> 6;
            const int c = cc & 63;
            const int k = kb + rr;
            const int qi = half, qj = 2 + half;
            const bool li = ((ent >> (kStepSlabShift + qi)) & 1) && k < n && k >= ks[qi];
            const bool lj = !diag && ((ent >> (kStepSlabShift + qj)) & 1) && k < n && k >= ks[qj];
            rI[e] = li ? *reinterpret_cast<const float4*>(xs[qi] + (int64_t)(k - ks[qi]) * kTile + c)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
            rJ[e] = lj ? *reinterpret_cast<const float4*>(xs[qj] + (int64_t)(k - ks[qj]) * kTile + c)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_step = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kSyrkKC / 8; ++e) {
            const int idx = threadIdx.x + 256 * e;
            const int rr = idx >> 5;
            const int cc = 4 * (idx & 31);
            *reinterpret_cast<float4*>(&sI[buf][rr * kWideLd + cc]) = rI[e];
            if (!diag) *reinterpret_cast<float4*>(&sJ[buf][rr * kWideLd + cc]) = rJ[e];
        }
    };

    const int nsteps = it.nsteps;
    if (nsteps > 0) {
        load_step(KS[0]);
        store_step(0);
    }
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        const int buf = st & 1;
        if (st + 1 < nsteps) load_step(KS[st + 1]);
        {
#pragma unroll
            for (int s = 0; s < kSyrkKC / 4; ++s) {
                const float* ai = &sI[buf][(4 * s + g) * kWideLd + 64 * wi + j];
                const float* bj = &(diag ? sI : sJ)[buf][(4 * s + g) * kWideLd + 64 * wj + j];
                float a[4], b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    a[t] = ai[16 * t];
                    b[t] = bj[16 * t];
                }
#pragma unroll
                for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = mfma_f32(a[ti], b[tj], acc[ti][tj]);
            }
        }
        if (st + 1 < nsteps) store_step(buf ^ 1);
        __syncthreads();
    }
    float* __restrict__ Ft = F + S.F_off + (int64_t)(it.I * (it.I + 1) / 2 + it.J) * kFTileElems;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Ft[(64 * wi + 16 * ti + 4 * g + r) * kSyrkTile + 64 * wj + 16 * tj + j] = acc[ti][tj][r];
}

__global__ __launch_bounds__(256) void syrk_tile_f32(
    const SubDev* __restrict__ subs, const TileDev* __restrict__ tiles,
    const SyrkItem* __restrict__ items, const int32_t* __restrict__ ksteps, const float* __restrict__ X,
    float* __restrict__ F)
{
    __shared__ __align__(16) char smem[kWideSmemF];
    const SyrkItem it = items[blockIdx.x];
    if (it.sub < 0) return;
    syrk_tile_item_f32(subs, tiles, it, ksteps, X, F, smem);
}

// ---------------------------------------------------------------------------
hipError_t launch_trsm(const DevTables& t, const int32_t* order, int64_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    if (t.X32) {
        if (t.trsm_merge)
            hipLaunchKernelGGL(trsm_stair_mixed<true>, dim3((unsigned)count), dim3(256), 0, stream, t.subs, t.tiles,
                               t.blocks, t.rows, t.visit, t.vrows, t.lval, t.lval32, t.piv, t.sgn, order, t.X32);
        else
            hipLaunchKernelGGL(trsm_stair_mixed<false>, dim3((unsigned)count), dim3(256), 0, stream, t.subs, t.tiles,
                               t.blocks, t.rows, t.visit, t.vrows, t.lval, t.lval32, t.piv, t.sgn, order, t.X32);
    } else {
        if (t.trsm_merge)
            hipLaunchKernelGGL(trsm_stair_f64<true>, dim3((unsigned)count), dim3(256), 0, stream, t.subs, t.tiles,
                               t.blocks, t.rows, t.visit, t.vrows, t.lval, t.piv, t.sgn, order, t.X);
        else
            hipLaunchKernelGGL(trsm_stair_f64<false>, dim3((unsigned)count), dim3(256), 0, stream, t.subs, t.tiles,
                               t.blocks, t.rows, t.visit, t.vrows, t.lval, t.piv, t.sgn, order, t.X);
    }
    return hipGetLastError();
}

hipError_t launch_syrk(const DevTables& t, const SyrkItem* items, int64_t ntile, int64_t nblock,
                       hipStream_t stream) {
    if (ntile > 0) {
        if (t.X32)
            hipLaunchKernelGGL(syrk_tile_f32, dim3((unsigned)ntile), dim3(256), 0, stream, t.subs, t.tiles, items,
                               t.ksteps, t.X32, t.F32);
        else
            hipLaunchKernelGGL(syrk_tile_f64, dim3((unsigned)ntile), dim3(256), 0, stream, t.subs, t.tiles, items,
                               t.ksteps, t.X, t.F);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nblock > 0) {
        if (t.X32)
            hipLaunchKernelGGL(syrk_block_f32, dim3((unsigned)nblock), dim3(256), 0, stream, t.subs, t.tiles,
                               items + ntile, t.ksteps, t.X32, t.F32);
        else
            hipLaunchKernelGGL(syrk_block_f64, dim3((unsigned)nblock), dim3(256), 0, stream, t.subs, t.tiles,
                               items + ntile, t.ksteps, t.X, t.F);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_assemble(const DevTables& t, hipStream_t stream, hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    if ((e = launch_trsm(t, t.tile_order, t.ntiles, stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], stream)) != hipSuccess) return e;
    if ((e = launch_syrk(t, t.syrk, t.nsyrk_tile, t.nsyrk - t.nsyrk_tile, stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], stream)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_convert_f32(const double* a, float* b, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(convert_f64_f32, dim3((unsigned)blocks), dim3(256), 0, stream, a, b, n);
    return hipGetLastError();
}

}  // namespace scasm
