// HIP kernels for gfx950 (CDNA4, wave64): the solution stage on the
// assembled F (explicit apply, Sec. 2.2 eq. (12); PCPG, Sec. 2.1 eq. (7))
// and the implicit apply with the factor (Sec. 2.2 eq. (11)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "device.hpp"
#include "kernels.hpp"

namespace scasm {

// ---------------------------------------------------------------------------
// Explicit apply q = F p (Sec. 2.2, eq. (12)) on the packed sorted F, FP64
// accumulation (FP32 or FP64 F).  Each stored lower tile T = F_s[I, J] is
// read once and used twice: pass 1, one workgroup per tile, writes
// u = T p_s[J] and v = T^T p_s[I] (p_s: p in sorted column order, gathered
// through pi; diagonal tiles are stored whole, v unused); pass 2, one
// workgroup per 128-row block K of a subdomain, sums u of (K, J <= K) and v
// of (I > K, K) in a fixed order and scatters the result to q in multiplier
// order.  Deterministic; reads F once, about half of the dense m x m.
// The partial sums of stored tile k live at part[(k - part_base) * 256]: the
// plan-owned buffer holds every tile (part_base 0); the fixed scratch array of
// the allocation-free apply holds one chunk of subdomains at a time.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void load8(const T* __restrict__ src, double (&t)[8]) {
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double2 d = reinterpret_cast<const double2*>(src)[e];
            t[2 * e] = d.x;
            t[2 * e + 1] = d.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float4 f = reinterpret_cast<const float4*>(src)[e];
            t[4 * e] = f.x;
            t[4 * e + 1] = f.y;
            t[4 * e + 2] = f.z;
            t[4 * e + 3] = f.w;
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void symv_tiles(
    const SubDev* __restrict__ subs, const SyrkItem* __restrict__ ftiles, const T* __restrict__ F,
    const int32_t* __restrict__ pi, const double* __restrict__ p, double* __restrict__ part, int64_t part_base)
{
    __shared__ double sp[2][kSyrkTile];                 // p_s of the tile's columns (J) and rows (I)
    __shared__ double su[kSyrkTile][17];                // row sums per group of 8 columns
    __shared__ double sv[kSyrkTile][17];                // column sums per group of 8 rows
    const SyrkItem it = ftiles[blockIdx.x];
    const SubDev S = subs[it.sub];
    const int tid = threadIdx.x;
    {
        const int half = tid >> 7;
        const int a = (half ? it.I : it.J) * kSyrkTile + (tid & 127);
        sp[half][tid & 127] = a < S.m ? p[S.dual_off + pi[S.col_off + a]] : 0.0;
    }
    __syncthreads();
    const int64_t tile = (int64_t)it.I * (it.I + 1) / 2 + it.J;
    const T* __restrict__ Ft = F + S.F_off + tile * kFTileElems;
    const int tr = tid >> 4;                            // rows 8 tr .. 8 tr + 7
    const int tc = tid & 15;                            // columns 8 tc .. 8 tc + 7
    double pj[8], u[8], v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        pj[c] = sp[0][8 * tc + c];
        u[c] = 0.0;
        v[c] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int row = 8 * tr + i;
        const double pr = sp[1][row];
        double t[8];
        load8(Ft + row * kSyrkTile + 8 * tc, t);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            u[i] += t[c] * pj[c];
            v[c] += t[c] * pr;
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        su[8 * tr + i][tc] = u[i];
        sv[8 * tc + i][tr] = v[i];
    }
    __syncthreads();
    const int k = tid & 127;
    double acc = 0.0;
    if (tid < 128) {
#pragma unroll
        for (int g = 0; g < 16; ++g) acc += su[k][g];
    } else {
#pragma unroll
        for (int g = 0; g < 16; ++g) acc += sv[k][g];
    }
    part[((S.ftile_off + tile - part_base) << 8) + tid] = acc;
}

__global__ __launch_bounds__(128) void symv_rows(
    const SubDev* __restrict__ subs, const int2* __restrict__ frows, const int32_t* __restrict__ pi,
    const double* __restrict__ part, int64_t part_base, double* __restrict__ q)
{
    const int2 it = frows[blockIdx.x];                  // (subdomain, row block K)
    const SubDev S = subs[it.x];
    const int K = it.y;
    const int r = threadIdx.x;
    const int nt = (S.m + kSyrkTile - 1) / kSyrkTile;
    const double* __restrict__ P = part + ((S.ftile_off - part_base) << 8);
    double y = 0.0;
    for (int J = 0; J <= K; ++J) y += P[(((int64_t)K * (K + 1) / 2 + J) << 8) + r];
    for (int I = K + 1; I < nt; ++I) y += P[(((int64_t)I * (I + 1) / 2 + K) << 8) + 128 + r];
    const int a = K * kSyrkTile + r;
    if (a < S.m) q[S.dual_off + pi[S.col_off + a]] = y;
}

// pass 1 over stored tiles [t0, t1), pass 2 over row blocks [r0, r1): the
// tiles of whole subdomains, partial sums at part[(k - t0) * 256]
static hipError_t apply_range(const DevTables& t, const double* p, double* q, double* part, int64_t t0, int64_t t1,
                              int64_t r0, int64_t r1, hipStream_t stream) {
    if (t1 <= t0) return hipSuccess;
    if (t.F32)
        hipLaunchKernelGGL(symv_tiles<float>, dim3((unsigned)(t1 - t0)), dim3(256), 0, stream, t.subs,
                           t.ftiles + t0, (const float*)t.F32, t.pi, p, part, t0);
    else
        hipLaunchKernelGGL(symv_tiles<double>, dim3((unsigned)(t1 - t0)), dim3(256), 0, stream, t.subs,
                           t.ftiles + t0, (const double*)t.F, t.pi, p, part, t0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(symv_rows, dim3((unsigned)(r1 - r0)), dim3(128), 0, stream, t.subs, t.frows + r0, t.pi,
                       (const double*)part, t0, q);
    return hipGetLastError();
}

hipError_t launch_apply(const DevTables& t, const double* p, double* q, hipStream_t stream, hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    if ((e = apply_range(t, p, q, t.part, 0, t.nftiles, 0, t.nfrows, stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Allocation-free explicit apply: the partial sums go to a fixed device array
// (one per GPU, for the life of the process) instead of the plan's buffer;
// the batch runs in chunks of whole subdomains whose stored tiles fit it, one
// chunk after the other on the caller's stream.  Every call on a GPU shares
// that GPU's array, so calls that overlap on one GPU race.  Nothing needs
// clearing: pass 1 writes every partial sum that pass 2 of its chunk reads.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kApplyScratchTiles * 256];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t apply_scratch_init(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;     // caller makes `device` current
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)ptr;
    }
    if (out) *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_apply_chunked(const DevTables& t, const ApplyChunk* chunks, int64_t nchunks, double* scratch_ptr,
                                const double* p, double* q, hipStream_t stream) {
    for (int64_t c = 0; c < nchunks; ++c) {
        const ApplyChunk& k = chunks[c];
        if (k.t1 - k.t0 > kApplyScratchTiles) return hipErrorInvalidValue;
        hipError_t e = apply_range(t, p, q, scratch_ptr, k.t0, k.t1, k.r0, k.r1, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Projected conjugate gradients on each subdomain's dual problem (Sec. 2.1,
// eq. (7), with e = 0 and the identity preconditioner), FP64 vectors; the
// per-subdomain scalars stay on the device.  One workgroup per subdomain.
//   lambda_0 = 0, r_0 = d, w_0 = P r_0, p_0 = w_0,  P = I - G (G^T G)^{-1} G^T
//   q = F p;  alpha = (w.w)/(p.q);  lambda += alpha p;  r -= alpha q
//   w' = P r;  beta = (w'.w')/(w.w);  p = w' + beta p
// ---------------------------------------------------------------------------
constexpr int kMaxKer = 8;

struct PcpgDev {
    const double* G;        // per subdomain m x k, column-major, at g_off
    const int64_t* g_off;
    const int32_t* kdim;
    const double* GtGinv;   // per subdomain k x k at 64 * sub
    double* r;
    double* w;
    double* pvec;
    double* q;
    double* ww;             // per subdomain w.w
    double* hist;           // (iters + 1) x nsub or null
    int32_t nsub;
};

__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) t += red[i];
    return t;
}

// w = r - G (G^T G)^{-1} G^T r over one subdomain; returns w.w
__device__ double project(const SubDev& S, const PcpgDev& D, int sub, const double* r, double* w, double* red,
                          double* su) {
    const int m = S.m;
    const int k = D.kdim[sub];
    const double* G = D.G + D.g_off[sub];
    for (int c = 0; c < k; ++c) {
        double t = 0.0;
        for (int i = threadIdx.x; i < m; i += 256) t += G[(int64_t)c * m + i] * r[i];
        t = block_sum(t, red);
        if (threadIdx.x == 0) su[c] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double u = 0.0;
        for (int c = 0; c < k; ++c) u += D.GtGinv[64 * sub + threadIdx.x * k + c] * su[c];
        su[kMaxKer + threadIdx.x] = u;
    }
    __syncthreads();
    double ww = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        double v = r[i];
        for (int c = 0; c < k; ++c) v -= G[(int64_t)c * m + i] * su[kMaxKer + c];
        w[i] = v;
        ww += v * v;
    }
    return block_sum(ww, red);
}

__global__ __launch_bounds__(256) void pcpg_init(const SubDev* __restrict__ subs, PcpgDev D,
                                                 const double* __restrict__ d, double* __restrict__ lambda) {
    __shared__ double red[4];
    __shared__ double su[2 * kMaxKer];
    const int sub = blockIdx.x;
    const SubDev S = subs[sub];
    const int64_t o = S.dual_off;
    for (int i = threadIdx.x; i < S.m; i += 256) {
        lambda[o + i] = 0.0;
        D.r[o + i] = d[o + i];
    }
    __syncthreads();
    const double ww = project(S, D, sub, D.r + o, D.w + o, red, su);
    for (int i = threadIdx.x; i < S.m; i += 256) D.pvec[o + i] = D.w[o + i];
    if (threadIdx.x == 0) {
        D.ww[sub] = ww;
        if (D.hist) D.hist[sub] = sqrt(ww);
    }
}

__global__ __launch_bounds__(256) void pcpg_step(const SubDev* __restrict__ subs, PcpgDev D,
                                                 double* __restrict__ lambda, int iter) {
    __shared__ double red[4];
    __shared__ double su[2 * kMaxKer];
    const int sub = blockIdx.x;
    const SubDev S = subs[sub];
    const int64_t o = S.dual_off;
    const int m = S.m;
    double* r = D.r + o;
    double* w = D.w + o;
    double* pv = D.pvec + o;
    const double* q = D.q + o;
    const double ww = D.ww[sub];
    double pq = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) pq += pv[i] * q[i];
    pq = block_sum(pq, red);
    const bool go = pq > 0.0 && ww > 0.0;       // converged (or breakdown): keep the iterate
    const double alpha = go ? ww / pq : 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        lambda[o + i] += alpha * pv[i];
        r[i] -= alpha * q[i];
    }
    __syncthreads();
    const double ww2 = go ? project(S, D, sub, r, w, red, su) : ww;
    const double beta = go ? ww2 / ww : 0.0;
    if (go)
        for (int i = threadIdx.x; i < m; i += 256) pv[i] = w[i] + beta * pv[i];
    if (threadIdx.x == 0) {
        D.ww[sub] = ww2;
        if (D.hist) D.hist[(int64_t)(iter + 1) * D.nsub + sub] = sqrt(ww2);
    }
}

hipError_t launch_pcpg(const DevTables& t, const PcpgArgs& a, hipStream_t stream, const ImplicitLevels* lvh,
                       const int64_t* xoff, double* xwork, int32_t nimpl) {
    PcpgDev D;
    D.G = a.G; D.g_off = a.g_off; D.kdim = a.kdim; D.GtGinv = a.GtGinv;
    D.r = a.r; D.w = a.w; D.pvec = a.p; D.q = a.q; D.ww = a.ww; D.hist = a.hist; D.nsub = a.nsub;
    if (a.nsub <= 0) return hipSuccess;
    hipLaunchKernelGGL(pcpg_init, dim3((unsigned)a.nsub), dim3(256), 0, stream, t.subs, D, a.d, a.lambda);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int it = 0; it < a.iters; ++it) {
        if ((e = launch_apply(t, a.p, a.q, stream, nullptr)) != hipSuccess) return e;
        if (lvh && (e = launch_apply_implicit(t, *lvh, xoff, xwork, a.p, a.q, nimpl, stream, nullptr)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(pcpg_step, dim3((unsigned)a.nsub), dim3(256), 0, stream, t.subs, D, a.lambda, it);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Implicit apply (Sec. 2.2, eq. (11)): q = B P^T L^{-T} L^{-1} P B^T p with the
// factor blocks, FP64.  x (n doubles per subdomain, workspace) holds P B^T p,
// then y = L^{-1} x, then z = L^{-T} y, in place.  The blocked triangular
// solves run level by level (planner: a block's forward level is one more
// than that of every block whose pruned rows reach it; its backward level one
// more than that of every block its own pruned rows lie in), one launch per
// level, one wavefront per block of all subdomains at that level:
//   forward, block b:   y_b = L_bb^{-1} (x_b - sum of the update entries of
//                       its rows), then u_b = L[R_b, b] y_b into the update
//                       buffer (parallel to the pruned-row lists); a row's
//                       entries are summed by its own thread in a fixed order
//                       (planner lists), no atomics
//   backward, block b:  z_b = L_bb^{-T} (y_b - L[R_b, b]^T z[R_b])
// The diagonal inverses are the ones the TRSM uses.  Repeated DOFs (several
// multipliers on one DOF) are summed by one thread per run of equal pivots.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tile_at(const double* __restrict__ At, int nks, int q, int k) {
    return At[((int64_t)(q >> 4) * nks + (k >> 2)) * 64 + (q & 15) + 16 * (k & 3)];
}

// Linv[r][k], k <= r (or within r's diagonal 16 x 16 tile), of a block's
// inverse diagonal: lower tiles only, tile (rt, ks) at 64 (2 rt (rt + 1) + ks)
__device__ __forceinline__ double linv_at(const double* __restrict__ Lv, int r, int k) {
    const int rt = r >> 4;
    return Lv[(2 * rt * (rt + 1) + (k >> 2)) * 64 + (r & 15) + 16 * (k & 3)];
}

// one 1024-thread workgroup per subdomain (x has n_i entries: ~30k on the
// 20^3 subdomains)
constexpr int kInitThreads = 1024;

__global__ __launch_bounds__(kInitThreads) void implicit_init(
    const SubDev* __restrict__ subs, const int32_t* __restrict__ piv, const int32_t* __restrict__ pi,
    const int8_t* __restrict__ sgn, const int64_t* __restrict__ xoff, const double* __restrict__ p,
    double* __restrict__ xwork, const int32_t* __restrict__ sub_list)
{
    const int sub = sub_list ? sub_list[blockIdx.x] : (int)blockIdx.x;
    const SubDev S = subs[sub];
    double* __restrict__ x = xwork + xoff[sub];
    const int32_t* __restrict__ pv = piv + S.col_off;
    const int32_t* __restrict__ pis = pi + S.col_off;
    const int8_t* __restrict__ sg = sgn + S.col_off;
    const double* __restrict__ ps = p + S.dual_off;
    for (int i = threadIdx.x; i < S.n; i += kInitThreads) x[i] = 0.0;
    __syncthreads();
    for (int a = threadIdx.x; a < S.m; a += kInitThreads) {
        if (a > 0 && pv[a - 1] == pv[a]) continue;
        double v = 0.0;
        for (int b = a; b < S.m && pv[b] == pv[a]; ++b) v += (double)sg[b] * ps[pis[b]];
        x[pv[a]] = v;
    }
}

// One block step per workgroup of kImplThreads threads: thread (part, r) =
// (tid / 64, tid % 64) works on row / column r and a 1/kImplParts share of
// each sum; partial sums meet in LDS in a fixed order.  The blocks of a level
// are few (the chain of one subdomain each), so each step spreads its short
// dependent sums over many threads.
constexpr int kImplThreads = 1024;
constexpr int kImplParts = kImplThreads / 64;
// factor tiles each wavefront has in flight in the off-diagonal products:
// 16 where a launch has fewer workgroups than compute units (the step's
// latency is the level's time), 8 on wide levels (two workgroups per CU
// share the memory system)
constexpr int kImplBatchNarrow = 16, kImplBatchWide = 8;
constexpr int64_t kImplNarrowBelow = 256;
constexpr int kImplSplit = 4;

__device__ __forceinline__ double sum_parts(const double (*sp)[64], int r) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kImplParts; ++k) v += sp[k][r];
    return v;
}

// forward step of block bd of subdomain S: x_b <- L_bb^{-1}(x_b - updates),
// then its updates L[R_b, b] x_b into its entries of ubuf
template <int NB>
__device__ __forceinline__ void implicit_fwd_block(
    const SubDev& S, const BlockDev& bd, const double* __restrict__ lval, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ rpos, const double* __restrict__ x, double* __restrict__ yo,
    double* __restrict__ ubuf, double (*sp)[64], double* sx, int g = 0, int G = 1)
{
    const double* __restrict__ L = lval + S.lval_off;
    const int tid = threadIdx.x;
    const int r = tid & 63;
    const int part = tid >> 6;
    const int w = bd.w;
    // x_b minus the update entries of its rows
    double v = 0.0;
    if (r < w) {
        const int row = bd.row0 + r;
        for (int e = rp[row] + part; e < rp[row + 1]; e += kImplParts) v -= ubuf[rpos[e]];
        if (part == 0) v += x[row];
    }
    sp[part][r] = v;
    __syncthreads();
    if (tid < 64) sx[tid] = sum_parts(sp, tid);
    __syncthreads();
    // y_b = L_bb^{-1} x_b: k split in kImplParts ranges of 4
    const double* __restrict__ Lv = L + bd.linv_off;
    double y = 0.0;
    if (r < w) {
        double a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = 4 * part + i <= r ? linv_at(Lv, r, 4 * part + i) : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (4 * part + i <= r) y += a[i] * sx[4 * part + i];
    }
    sp[part][r] = y;
    __syncthreads();
    if (tid < 64) {
        const double yb = sum_parts(sp, tid);
        sx[tid] = tid < w ? yb : 0.0;
        if (g == 0 && tid < w) yo[bd.row0 + tid] = yb;   // one writer of the G copies
    }
    __syncthreads();
    // u_b = L[R_b, b] y_b: wavefront `part` takes row tiles part, part +
    // kImplParts, ...; lane l the products L[16 t + l % 16, 4 s + l / 16]
    // y[4 s + l / 16] over the k-slices s of row tile t, each wavefront load
    // one whole 512-byte A tile, NB in flight at a time; then the four
    // lanes of a row combine (y is zero past w, the tiles' padding is zero)
    const double* __restrict__ At = L + bd.aoff;
    const int nks = (w + 3) >> 2;
    const int nrt = (bd.nbelow + 15) >> 4;
    double* __restrict__ u = ubuf + S.rows_off + bd.rows_off;
    for (int t = part + kImplParts * g; t < nrt; t += kImplParts * G) {
        const double* __restrict__ Tt = At + (int64_t)t * nks * 64 + r;
        double acc = 0.0;
        for (int s0 = 0; s0 < nks; s0 += NB) {
            double a[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) a[i] = s0 + i < nks ? Tt[(s0 + i) * 64] : 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (s0 + i < nks) acc += a[i] * sx[4 * (s0 + i) + (r >> 4)];
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        if (r < 16 && 16 * t + r < bd.nbelow) u[16 * t + r] = acc;
    }
}

template <int NB>
__global__ __launch_bounds__(kImplThreads) void implicit_fwd(
    const SubDev* __restrict__ subs, const BlockDev* __restrict__ blocks, const double* __restrict__ lval,
    const int64_t* __restrict__ rptr_off, const int32_t* __restrict__ rptr, const int32_t* __restrict__ rpos,
    const int2* __restrict__ items, const int64_t* __restrict__ xoff, double* __restrict__ xwork,
    double* __restrict__ ywork, double* __restrict__ ubuf, int G)
{
    __shared__ double sp[kImplParts][64];
    __shared__ double sx[64];
    const int2 it = items[blockIdx.x / G];
    const SubDev S = subs[it.x];
    const BlockDev bd = blocks[S.blk_off + it.y];
    implicit_fwd_block<NB>(S, bd, lval, rptr + rptr_off[it.x], rpos, xwork + xoff[it.x], ywork + xoff[it.x], ubuf,
                           sp, sx, (int)(blockIdx.x % G), G);
}

// backward step of block bd: z_b <- L_bb^{-T}(y_b - L[R_b, b]^T z[R_b])
template <int NB>
__device__ __forceinline__ void implicit_bwd_block(
    const SubDev& S, const BlockDev& bd, const int32_t* __restrict__ rows, const double* __restrict__ lval,
    const double* __restrict__ yi, double* __restrict__ x, double (*sp)[64], double* sz, double* sv)
{
    const double* __restrict__ L = lval + S.lval_off;
    const int32_t* __restrict__ rw = rows + S.rows_off + bd.rows_off;
    const int tid = threadIdx.x;
    const int r = tid & 63;
    const int part = tid >> 6;
    const int w = bd.w, nb = bd.nbelow, nks = (w + 3) >> 2;
    const double* __restrict__ At = L + bd.aoff;
    // y_b - L[R_b, b]^T z[R_b]: pruned rows in groups of kImplThreads;
    // wavefront `part` takes k-slice `part` (columns 4 part .. 4 part + 3),
    // lane l the products L[16 t + l % 16, 4 part + l / 16] z[16 t + l % 16]
    // over the row tiles t: each wavefront load is one whole 512-byte A tile,
    // NB in flight at a time.  Rows past nb read the tiles' zero padding
    // against zero z entries.
    double acc = 0.0;
    for (int c0 = 0; c0 < nb; c0 += kImplThreads) {
        __syncthreads();
        sz[tid] = c0 + tid < nb ? x[rw[c0 + tid]] : 0.0;   // z of the pruned rows: final
        __syncthreads();
        if (part < nks) {
            const int nrt = (min(kImplThreads, nb - c0) + 15) >> 4;
            const double* __restrict__ Ts = At + ((int64_t)(c0 >> 4) * nks + part) * 64 + r;
            for (int t0 = 0; t0 < nrt; t0 += NB) {
                double a[NB];
#pragma unroll
                for (int i = 0; i < NB; ++i) a[i] = t0 + i < nrt ? Ts[(int64_t)(t0 + i) * nks * 64] : 0.0;
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (t0 + i < nrt) acc += a[i] * sz[16 * (t0 + i) + (r & 15)];
            }
        }
    }
    // column 4 part + l / 16: the sum over its 16 lanes
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 8, 64);
    if (part < nks && (r & 15) == 0 && 4 * part + (r >> 4) < w)
        sv[4 * part + (r >> 4)] = yi[bd.row0 + 4 * part + (r >> 4)] - acc;
    __syncthreads();
    // z_b = L_bb^{-T} v: k split in kImplParts ranges of 4
    const double* __restrict__ Lv = L + bd.linv_off;
    double z = 0.0;
    if (r < w) {
        double a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * part + i;
            a[i] = k >= r && k < w ? linv_at(Lv, k, r) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * part + i;
            if (k >= r && k < w) z += a[i] * sv[k];
        }
    }
    sp[part][r] = z;
    __syncthreads();
    if (tid < w) x[bd.row0 + tid] = sum_parts(sp, tid);
}

template <int NB>
__global__ __launch_bounds__(kImplThreads) void implicit_bwd(
    const SubDev* __restrict__ subs, const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows,
    const double* __restrict__ lval, const int2* __restrict__ items, const int64_t* __restrict__ xoff,
    const double* __restrict__ ywork, double* __restrict__ xwork)
{
    __shared__ double sp[kImplParts][64];
    __shared__ double sz[kImplThreads];
    __shared__ double sv[64];
    const int2 it = items[blockIdx.x];
    const SubDev S = subs[it.x];
    const BlockDev bd = blocks[S.blk_off + it.y];
    implicit_bwd_block<NB>(S, bd, rows, lval, ywork + xoff[it.x], xwork + xoff[it.x], sp, sz, sv);
}

// Both sweeps of one subdomain in one workgroup: its blocks in increasing
// order (forward) and decreasing order (backward) are dependency orders, and
// a workgroup barrier (a workgroup-scope release / acquire of the global
// writes) separates consecutive blocks; no launch per level.
__global__ __launch_bounds__(kImplThreads) void implicit_sweeps(
    const SubDev* __restrict__ subs, const BlockDev* __restrict__ blocks, const int32_t* __restrict__ rows,
    const double* __restrict__ lval, const int64_t* __restrict__ rptr_off, const int32_t* __restrict__ rptr,
    const int32_t* __restrict__ rpos, const int64_t* __restrict__ xoff, double* __restrict__ xwork,
    double* __restrict__ ywork, double* __restrict__ ubuf, const int32_t* __restrict__ sub_list)
{
    __shared__ double sp[kImplParts][64];
    __shared__ double sx[64];
    __shared__ double sz[kImplThreads];
    const int sub = sub_list ? sub_list[blockIdx.x] : (int)blockIdx.x;
    const SubDev S = subs[sub];
    double* __restrict__ x = xwork + xoff[sub];
    double* __restrict__ y = ywork + xoff[sub];
    const int32_t* __restrict__ rp = rptr + rptr_off[sub];
    for (int b = 0; b < S.nblocks; ++b) {
        const BlockDev bd = blocks[S.blk_off + b];
        implicit_fwd_block<kImplBatchNarrow>(S, bd, lval, rp, rpos, x, y, ubuf, sp, sx);
        __syncthreads();
    }
    for (int b = S.nblocks - 1; b >= 0; --b) {
        const BlockDev bd = blocks[S.blk_off + b];
        implicit_bwd_block<kImplBatchNarrow>(S, bd, rows, lval, y, x, sp, sz, sx);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kInitThreads) void implicit_gather(
    const SubDev* __restrict__ subs, const int32_t* __restrict__ piv, const int32_t* __restrict__ pi,
    const int8_t* __restrict__ sgn, const int64_t* __restrict__ xoff, const double* __restrict__ xwork,
    double* __restrict__ q, const int32_t* __restrict__ sub_list)
{
    const int sub = sub_list ? sub_list[blockIdx.x] : (int)blockIdx.x;
    const SubDev S = subs[sub];
    const double* __restrict__ x = xwork + xoff[sub];
    for (int a = threadIdx.x; a < S.m; a += kInitThreads)
        q[S.dual_off + pi[S.col_off + a]] = (double)sgn[S.col_off + a] * x[piv[S.col_off + a]];
}

hipError_t launch_implicit_init(const DevTables& t, const int64_t* xoff, double* xwork, const double* p,
                                const int32_t* sub_list, int32_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(implicit_init, dim3((unsigned)count), dim3(kInitThreads), 0, stream, t.subs, t.piv, t.pi, t.sgn,
                       xoff, p, xwork, sub_list);
    return hipGetLastError();
}

hipError_t launch_implicit_sweeps(const DevTables& t, const ImplicitLevels& lv, const int64_t* xoff, double* xwork,
                                  int32_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    // every table and workspace the sweeps dereference must be in place
    if (!xoff || !xwork || !lv.ywork || !lv.ubuf || !lv.rptr_off || !lv.rptr || !lv.rpos) return hipErrorInvalidValue;
    if (!lv.per_subdomain && ((lv.fw_off.size() > 1 && !lv.fw_items) || (lv.bw_off.size() > 1 && !lv.bw_items)))
        return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (lv.per_subdomain) {
        hipLaunchKernelGGL(implicit_sweeps, dim3((unsigned)count), dim3(kImplThreads), 0, stream, t.subs, t.blocks,
                           t.rows, t.lval, lv.rptr_off, lv.rptr, lv.rpos, xoff, xwork, lv.ywork, lv.ubuf, lv.subs);
        return hipGetLastError();
    }
    for (size_t l = 0; l + 1 < lv.fw_off.size(); ++l) {
        const int64_t cnt = lv.fw_off[l + 1] - lv.fw_off[l];
        if (cnt <= 0) continue;
        // narrow levels: kImplSplit workgroups per block, each repeating the
        // update sums and the diagonal product and taking every kImplSplit-th
        // group of row tiles of the product below
        if (cnt < kImplNarrowBelow)
            hipLaunchKernelGGL(implicit_fwd<kImplBatchNarrow>, dim3((unsigned)(cnt * kImplSplit)), dim3(kImplThreads),
                               0, stream, t.subs, t.blocks, t.lval, lv.rptr_off, lv.rptr, lv.rpos,
                               lv.fw_items + lv.fw_off[l], xoff, xwork, lv.ywork, lv.ubuf, kImplSplit);
        else
            hipLaunchKernelGGL(implicit_fwd<kImplBatchWide>, dim3((unsigned)cnt), dim3(kImplThreads), 0, stream,
                               t.subs, t.blocks, t.lval, lv.rptr_off, lv.rptr, lv.rpos, lv.fw_items + lv.fw_off[l],
                               xoff, xwork, lv.ywork, lv.ubuf, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (size_t l = 0; l + 1 < lv.bw_off.size(); ++l) {
        const int64_t cnt = lv.bw_off[l + 1] - lv.bw_off[l];
        if (cnt <= 0) continue;
        if (cnt < kImplNarrowBelow)
            hipLaunchKernelGGL(implicit_bwd<kImplBatchNarrow>, dim3((unsigned)cnt), dim3(kImplThreads), 0, stream,
                               t.subs, t.blocks, t.rows, t.lval, lv.bw_items + lv.bw_off[l], xoff, lv.ywork,
                               xwork);
        else
            hipLaunchKernelGGL(implicit_bwd<kImplBatchWide>, dim3((unsigned)cnt), dim3(kImplThreads), 0, stream,
                               t.subs, t.blocks, t.rows, t.lval, lv.bw_items + lv.bw_off[l], xoff, lv.ywork,
                               xwork);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_implicit_gather(const DevTables& t, const int64_t* xoff, const double* xwork, double* q,
                                  const int32_t* sub_list, int32_t count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(implicit_gather, dim3((unsigned)count), dim3(kInitThreads), 0, stream, t.subs, t.piv, t.pi,
                       t.sgn, xoff, xwork, q, sub_list);
    return hipGetLastError();
}

hipError_t launch_apply_implicit(const DevTables& t, const ImplicitLevels& lv, const int64_t* xoff, double* xwork,
                                 const double* p, double* q, int32_t count, hipStream_t stream, hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    if ((e = launch_implicit_init(t, xoff, xwork, p, lv.subs, count, stream)) != hipSuccess) return e;
    if ((e = launch_implicit_sweeps(t, lv, xoff, xwork, count, stream)) != hipSuccess) return e;
    if ((e = launch_implicit_gather(t, xoff, xwork, q, lv.subs, count, stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace scasm
