// Kernel launchers (host side) over the device tables of a plan.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "device.hpp"

namespace scasm {

constexpr int kNumTimed = 5;   // timed kernels: TRSM, SYRK, apply, implicit apply, overlapped assembly

struct DevTables {
    const SubDev* subs = nullptr;
    const TileDev* tiles = nullptr;
    const BlockDev* blocks = nullptr;
    const int32_t* rows = nullptr;
    const int32_t* visit = nullptr;        // blocks visited per TRSM tile (TileDev::visit_off)
    const int32_t* ksteps = nullptr;       // SYRK k-steps per item (SyrkItem::step_off)
    const uint64_t* vrows = nullptr;       // per visit: rows of the block on the tile's paths
    const double* lval = nullptr;
    const float* lval32 = nullptr;
    const int32_t* piv = nullptr;
    const int32_t* pi = nullptr;
    const int8_t* sgn = nullptr;
    const SyrkItem* syrk = nullptr;
    const int32_t* tile_order = nullptr;   // TRSM workgroup -> tile index (-1 = idle)
    double* X = nullptr;
    float* X32 = nullptr;
    double* F = nullptr;
    float* F32 = nullptr;
    const SyrkItem* ftiles = nullptr;      // stored F tiles (subdomain order): symmetric apply pass 1
    const int2* frows = nullptr;           // (subdomain, 128-row block): symmetric apply pass 2
    double* part = nullptr;                // 256 partial sums per stored F tile
    int64_t ntiles = 0;          // TRSM workgroups (length of tile_order)
    bool trsm_merge = false;     // TRSM with the merged pairs of BlockDev::flags
    int64_t nsyrk = 0;           // SYRK workgroups (items with sub < 0 are idle)
    int64_t nsyrk_tile = 0;      // the first nsyrk_tile of them are 128 x 128 tiles, the rest 64 x 64 blocks
    int64_t nftiles = 0;
    int64_t nfrows = 0;
};

// Assembly kernels; FP64, or mixed precision when t.X32 is set (FP64
// diagonal solves, FP32 X / updates / SYRK and FP32 F).
//   launch_trsm: TRSM workgroups over `order[0, count)` (tile indices, -1 idle)
//   launch_syrk: SYRK workgroups over `items[0, count)` (sub < 0 idle)
//   launch_assemble: all tiles, then all SYRK items, on one stream; optional
//     events ev[2k] before and ev[2k+1] after kernel k (0 = TRSM, 1 = SYRK).
hipError_t launch_trsm(const DevTables& t, const int32_t* order, int64_t count, hipStream_t stream);
// SYRK over items[0, ntile) (128 x 128 tiles) then items[ntile, ntile + nblock)
// (64 x 64 blocks).
hipError_t launch_syrk(const DevTables& t, const SyrkItem* items, int64_t ntile, int64_t nblock,
                       hipStream_t stream);
hipError_t launch_assemble(const DevTables& t, hipStream_t stream, hipEvent_t* ev);

// FP64 factor -> FP32 copy (mixed precision).
hipError_t launch_convert_f32(const double* a, float* b, int64_t n, hipStream_t stream);

struct PcpgArgs {
    const double* G;        // concatenated m_i x k_i column-major blocks
    const int64_t* g_off;   // [nsub] offsets into G
    const int32_t* kdim;    // [nsub] kernel dimension k_i (<= 8)
    const double* GtGinv;   // [nsub][64] (G^T G)^{-1}, k_i x k_i row-major
    const double* d;        // right-hand side (dual layout)
    double* lambda;         // solution (dual layout)
    double *r, *w, *p, *q;  // workspace (dual layout)
    double* ww;             // [nsub]
    double* hist;           // [(iters + 1) * nsub] or null
    int32_t nsub;
    int32_t iters;
};

struct ImplicitLevels;
// Projected CG on every subdomain, `iters` iterations: F applied explicitly
// to the assembled subdomains, and, when lvh is given, with the factor to the
// nimpl subdomains of lvh->subs (workspace xwork at xoff).
hipError_t launch_pcpg(const DevTables& t, const PcpgArgs& a, hipStream_t stream, const ImplicitLevels* lvh,
                       const int64_t* xoff, double* xwork, int32_t nimpl);

// Level schedule of the blocked triangular solves of the implicit apply:
// items (subdomain, block) grouped by level (host offsets, levels run in
// order); per row of a subdomain (rptr at rptr_off[sub], CSR) the positions
// in the row array where it is a pruned row: its entries in the update
// buffer ubuf, which runs parallel to the row array.
struct ImplicitLevels {
    const int2* fw_items = nullptr;
    const int2* bw_items = nullptr;
    const int64_t* rptr_off = nullptr;
    const int32_t* rptr = nullptr;
    const int32_t* rpos = nullptr;
    double* ubuf = nullptr;
    // y = L^{-1} x of the forward sweep (n_i doubles per subdomain at the
    // xwork offsets): kept apart from x so that several workgroups of one
    // forward block step read x while one of them writes y
    double* ywork = nullptr;
    std::vector<int64_t> fw_off, bw_off;
    // true: one workgroup per subdomain runs both sweeps block by block (the
    // block DAGs are near chains); false: one launch per level
    bool per_subdomain = false;
    // the subdomains covered (device list; null = all, in index order)
    const int32_t* subs = nullptr;
};

// Implicit apply q = B P^T L^{-T} L^{-1} P B^T p; xwork holds n_i doubles per
// subdomain at xoff[i]; optional events ev[0] before, ev[1] after.  It is the
// three launches below in order: x = P B^T p (init), the two blocked
// triangular sweeps on x in place (they read no caller pointer, so a captured
// graph of them stays valid for any p and q), q = B P^T x (gather).
// `count` subdomains: those of `sub_list` / lv.subs, or 0 .. count - 1 when
// the list is null.
hipError_t launch_implicit_init(const DevTables& t, const int64_t* xoff, double* xwork, const double* p,
                                const int32_t* sub_list, int32_t count, hipStream_t stream);
hipError_t launch_implicit_sweeps(const DevTables& t, const ImplicitLevels& lv, const int64_t* xoff, double* xwork,
                                  int32_t count, hipStream_t stream);
hipError_t launch_implicit_gather(const DevTables& t, const int64_t* xoff, const double* xwork, double* q,
                                  const int32_t* sub_list, int32_t count, hipStream_t stream);
hipError_t launch_apply_implicit(const DevTables& t, const ImplicitLevels& lv, const int64_t* xoff, double* xwork,
                                 const double* p, double* q, int32_t count, hipStream_t stream, hipEvent_t* ev);

// q = F p for every subdomain (FP32 F when t.F32 is set, else FP64 F), two
// passes over the packed sorted F; optional events ev[0] before, ev[1] after.
hipError_t launch_apply(const DevTables& t, const double* p, double* q, hipStream_t stream, hipEvent_t* ev);

// Allocation-free explicit apply.  Its partial sums live in a fixed device
// array of kApplyScratchTiles stored tiles (256 doubles each: 32 MiB), one per
// GPU for the life of the process.
constexpr int64_t kApplyScratchTiles = 16384;
// largest m whose nst (nst + 1) / 2 stored tiles (nst = ceil(m / 128)) fit
constexpr int32_t kApplyMaxM = 180 * kSyrkTile;
static_assert(180 * 181 / 2 <= kApplyScratchTiles && 181 * 182 / 2 > kApplyScratchTiles, "kApplyMaxM");
constexpr int kMaxDevices = 64;
// Whole subdomains whose stored tiles [t0, t1) fit the array; their row
// blocks [r0, r1) (h_frows order).
struct ApplyChunk {
    int64_t t0, t1, r0, r1;
};
// Looks up (once per device, with `device` current) the device address of
// the array; *out receives it.  Thread-safe.
hipError_t apply_scratch_init(int device, double** out);
// q = F p chunk by chunk on `stream`, partial sums in `scratch_ptr` (from
// apply_scratch_init); no allocation.
hipError_t launch_apply_chunked(const DevTables& t, const ApplyChunk* chunks, int64_t nchunks, double* scratch_ptr,
                                const double* p, double* q, hipStream_t stream);

}  // namespace scasm
