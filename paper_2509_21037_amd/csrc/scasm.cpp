// C ABI of libscasm.so (declared in include/scasm.h).
#include "scasm.h"
#include "scasm_host.h"

#include <hip/hip_runtime.h>
#include <omp.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device.hpp"
#include "kernels.hpp"
#include "planner.hpp"

using namespace scasm;

namespace {

thread_local std::string g_last_error;

sc_status_t fail(sc_status_t st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

SubdomainInput to_input(const sc_subdomain_desc_t& d) {
    SubdomainInput in;
    in.n = d.n;
    in.rowptr = d.kreg_rowptr;
    in.col = d.kreg_col;
    in.m = d.m;
    in.dof = d.bt_dof;
    in.sign = d.bt_sign;
    in.perm = d.perm;
    in.coords = d.coords;
    in.dim = d.dim;
    in.dofs_per_node = d.dofs_per_node > 0 ? d.dofs_per_node : 1;
    return in;
}

// Plans one subdomain.  With lower_only the caller's CSR holds only the
// entries on and below the diagonal (col <= row): the pattern is mirrored for
// the ordering and the symbolic factorisation, and the map from CSR entries
// to factor slots is folded back onto the caller's entries, so sc_factor
// takes the caller's (lower) value arrays unchanged.
std::string plan_subdomain(const sc_subdomain_desc_t& d, const PlanOptions& po, bool lower_only, SubPlan& sp,
                           int& code) {
    SubdomainInput in = to_input(d);
    if (!lower_only) return build_plan(in, po, sp, code);
    code = 1;
    if (d.n <= 0 || !d.kreg_rowptr || !d.kreg_col) return "K_reg pattern missing";
    const int32_t n = d.n;
    if (d.kreg_rowptr[0] != 0) return "rowptr[0] must be 0";
    std::vector<int64_t> cnt(n + 1, 0);
    for (int32_t r = 0; r < n; ++r) {
        if (d.kreg_rowptr[r + 1] < d.kreg_rowptr[r]) return "rowptr not monotone";
        for (int64_t p = d.kreg_rowptr[r]; p < d.kreg_rowptr[r + 1]; ++p) {
            const int32_t c = d.kreg_col[p];
            if (c < 0 || c >= n) return "column index out of range";
            if (c > r) return "lower_only_csr: entry above the diagonal in row " + std::to_string(r);
            ++cnt[r + 1];
            if (c != r) ++cnt[c + 1];
        }
    }
    for (int32_t r = 0; r < n; ++r) cnt[r + 1] += cnt[r];
    std::vector<int64_t> rowptr(cnt.begin(), cnt.end());
    std::vector<int32_t> col((size_t)cnt[n]);
    std::vector<int64_t> src((size_t)cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t r = 0; r < n; ++r)
        for (int64_t p = d.kreg_rowptr[r]; p < d.kreg_rowptr[r + 1]; ++p) {
            const int32_t c = d.kreg_col[p];
            col[fill[r]] = c;
            src[fill[r]++] = p;
            if (c != r) {
                col[fill[c]] = r;
                src[fill[c]++] = p;
            }
        }
    in.rowptr = rowptr.data();
    in.col = col.data();
    std::string err = build_plan(in, po, sp, code);
    if (!err.empty()) return err;
    // each caller entry has exactly one mirrored copy on the stored (lower,
    // permuted) side; fold its slot back
    std::vector<int64_t> kmap((size_t)d.kreg_rowptr[n], -1);
    for (size_t e = 0; e < sp.kmap.size(); ++e)
        if (sp.kmap[e] >= 0) kmap[(size_t)src[e]] = sp.kmap[e];
    sp.kmap.swap(kmap);
    return "";
}

// Fills `po` from the ABI options; returns "" or an error message.
std::string to_plan_options(const sc_options_t& o, PlanOptions& po) {
    if (o.precision != SC_PREC_FP64 && o.precision != SC_PREC_MIXED) return "unknown precision";
    if (o.panel_width < 0 || o.relax_width < 0 || o.leaf_nodes < 0 || o.n_threads < 0)
        return "negative option";
    if (o.assembly_kernels < 0 || o.assembly_kernels > 2) return "assembly_kernels must be 0, 1 or 2";
    if (o.panel_width) po.panel_width = o.panel_width;
    if (po.panel_width > kMaxPanel || po.panel_width < 16) return "panel_width must be in [16, 64]";
    if (o.relax_width) po.relax_width = o.relax_width;
    if (o.leaf_nodes) po.leaf_nodes = o.leaf_nodes;
    po.staircase = o.disable_staircase ? 0 : 1;
    po.reach = o.disable_reach ? 0 : 1;
    if (o.block_split < 0 || o.block_split > 1) return "block_split must be 0 or 1";
    if (o.arena_cap_bytes < 0) return "arena_cap_bytes must be >= 0";
    if (o.select_iters < 0) return "select_iters must be >= 0";
    if (o.lower_only_csr < 0 || o.lower_only_csr > 1) return "lower_only_csr must be 0 or 1";
    if (o.syrk_kind < 0 || o.syrk_kind > 2) return "syrk_kind must be 0, 1 or 2";
    if (o.disable_pair_merge < 0 || o.disable_pair_merge > 1) return "disable_pair_merge must be 0 or 1";
    for (int k = 0; k < 3; ++k)
        if (!(o.select_model[k] >= 0.0f)) return "select_model rates must be >= 0";
    if (o.ntune_classes < 0 || (o.ntune_classes > 0 && !o.tune_classes)) return "bad tune_classes";
    for (int32_t c = 0; c < o.ntune_classes; ++c) {
        const sc_tune_class_t& k = o.tune_classes[c];
        if (k.n_lo < 0 || k.n_hi < k.n_lo) return "tune class: bad n range";
        if (k.panel_width != 0 && (k.panel_width < 16 || k.panel_width > kMaxPanel))
            return "tune class: panel_width must be 0 or in [16, 64]";
        if (k.block_split < -1 || k.block_split > 1) return "tune class: block_split must be -1, 0 or 1";
        if (k.syrk_kind < 0 || k.syrk_kind > 2) return "tune class: syrk_kind must be 0, 1 or 2";
    }
    po.block_split = o.block_split;
    return "";
}

// Per-subdomain explicit / implicit selection (select_iters): default rates
// measured on MI355X -- structural assembly TFLOP/s (FP64, mixed), explicit
// apply GB/s over the stored F, implicit apply GB/s over the two sweeps' 16
// bytes per factor entry.
constexpr double kSelectAsmTflops64 = 45.6;
constexpr double kSelectAsmTflopsMixed = 75.7;
constexpr double kSelectExplGBps = 5800.0;
constexpr double kSelectImplGBps = 3190.0;

// Share of a batch's TRSM pruned-row updates the merged pairs must save for
// the merge-capable TRSM kernel to be launched (the 12^3 heat batch saves 5%
// and ran 2% slower with it, the uneven elasticity batch 4% faster, the 20^3
// batch, 36% saved, 12% faster).
constexpr double kMergeMinShare = 0.10;

struct Prediction {
    double t_asm_ms = 0, t_expl_ms = 0, t_impl_ms = 0, n_star = 0;
};

// t_asm = structural flops / assembly rate; t_expl = stored F bytes / apply
// rate; t_impl = 16 nnz(L) / implicit rate; n* = t_asm / (t_impl - t_expl).
Prediction predict(const SubPlan& sp, bool mixed, const sc_options_t& o) {
    const double r_asm = o.select_model[0] > 0 ? o.select_model[0] : (mixed ? kSelectAsmTflopsMixed : kSelectAsmTflops64);
    const double r_expl = o.select_model[1] > 0 ? o.select_model[1] : kSelectExplGBps;
    const double r_impl = o.select_model[2] > 0 ? o.select_model[2] : kSelectImplGBps;
    const double nst = (double)((sp.m + kSyrkTile - 1) / kSyrkTile);
    Prediction q;
    q.t_asm_ms = (sp.trsm_reach + sp.syrk_reach) / (r_asm * 1e12) * 1e3;
    q.t_expl_ms = nst * (nst + 1) / 2 * kFTileElems * (mixed ? 4.0 : 8.0) / (r_expl * 1e9) * 1e3;
    q.t_impl_ms = 16.0 * (double)sp.nnzL / (r_impl * 1e9) * 1e3;
    q.n_star = q.t_impl_ms > q.t_expl_ms ? q.t_asm_ms / (q.t_impl_ms - q.t_expl_ms) : HUGE_VAL;
    return q;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? SC_ERR_OOM : SC_ERR_DEVICE,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t count = 0;
    hipError_t alloc(size_t n) {
        count = n;
        if (n == 0) return hipSuccess;
        return hipMalloc((void**)&p, n * sizeof(T));
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        count = 0;
    }
};

}  // namespace

struct sc_plan_s {
    int32_t nsub = 0;
    sc_options_t opt{};
    PlanOptions popt{};
    int device = 0;
    std::vector<SubPlan> plans;
    std::vector<int64_t> kval_count;          // CSR entries per subdomain
    // host mirrors of the tables
    std::vector<SubDev> h_subs;
    std::vector<TileDev> h_tiles;
    std::vector<BlockDev> h_blocks;
    std::vector<int32_t> h_visit;               // TRSM visit lists of all tiles
    std::vector<uint64_t> h_vrows;              // per visit: the block's rows on the paths
    std::vector<int32_t> h_ksteps;              // SYRK k-step lists of all items
    std::vector<SyrkItem> h_syrk;               // interleaved over XCDs, idle items sub = -1
    std::vector<int32_t> h_tile_order;          // TRSM workgroup -> tile (-1 idle)
    // overlapped assembly: groups of subdomains (every XCD's list cut into
    // kOverlapGroups consecutive parts), per group a TRSM order and SYRK list
    std::vector<int32_t> h_tile_order_g;
    std::vector<SyrkItem> h_syrk_g;
    std::vector<int64_t> g_toff, g_tcnt, g_soff, g_stile, g_sblock;
    // the same groups for the pipelined preprocessing (sc_preprocess): their
    // subdomains (g_sub[g_sub_off[g] .. g_sub_off[g + 1])) and factor values,
    // which are laid out group after group: [g_lval[g], g_lval[g + 1])
    std::vector<int32_t> g_sub;
    std::vector<int64_t> g_sub_off, g_lval;
    int64_t nsyrk_tile = 0;                     // h_syrk: 128 x 128 tiles first, then 64 x 64 blocks
    std::vector<SyrkItem> h_ftiles;             // stored F tiles, subdomain order (apply pass 1)
    std::vector<int2> h_frows;                  // (subdomain, 128-row block) (apply pass 2)
    int64_t nval_total = 0, nrows_total = 0, ncol_total = 0, X_total = 0, F_total = 0, dual_total = 0;
    double* h_lval = nullptr;                 // pinned
    // device
    DevBuf<SubDev> d_subs;
    DevBuf<TileDev> d_tiles;
    DevBuf<BlockDev> d_blocks;
    DevBuf<SyrkItem> d_syrk;
    DevBuf<int32_t> d_tile_order;
    DevBuf<int32_t> d_tile_order_g;
    DevBuf<SyrkItem> d_syrk_g;
    hipStream_t aux = nullptr;                  // second stream of the overlapped assembly
    std::vector<hipEvent_t> ov_events;          // one per group + join
    DevBuf<SyrkItem> d_ftiles;
    DevBuf<int2> d_frows;
    DevBuf<double> d_part;                      // apply partial sums, 256 per stored F tile
    // allocation-free apply: chunks of whole subdomains whose stored tiles fit
    // the fixed scratch array, that array's device address on this plan's
    // device, and the first subdomain too large for it (-1: none)
    std::vector<ApplyChunk> h_chunks;
    double* scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    int32_t noalloc_too_big = -1;
    DevBuf<int32_t> d_rows, d_piv, d_pi, d_visit, d_ksteps;
    DevBuf<uint64_t> d_vrows;
    DevBuf<int8_t> d_sgn;
    DevBuf<double> d_lval, d_X, d_F;
    DevBuf<float> d_lval32, d_X32, d_F32;
    DevBuf<double> d_xwork, d_ywork;          // implicit apply: n_i doubles per subdomain each
    DevBuf<int64_t> d_xoff;
    // implicit apply level schedule (built with the workspace, on first use)
    DevBuf<int2> d_ifw, d_ibw;
    DevBuf<int64_t> d_rptr_off;
    DevBuf<int32_t> d_rptr, d_rpos;
    DevBuf<double> d_ubuf;
    ImplicitLevels ilv;
    // the same schedule restricted to the subdomains applied implicitly in
    // sc_apply / sc_pcpg (select_iters)
    DevBuf<int2> d_ifw_h, d_ibw_h;
    DevBuf<int32_t> d_impl_list;
    ImplicitLevels ilv_h;
    bool mixed = false;
    bool factored = false, assembled = false;
    // temporary-memory waves (arena_cap_bytes > 0): X elements the cap holds;
    // the groups are then waves that reuse one X buffer one after the other
    int64_t arena_elems = 0;
    std::vector<int32_t> syrk_kind;             // per subdomain: 0 by size, 1 blocks, 2 tiles
    // the TRSM kernel with the merged pairs: when they save at least
    // kMergeMinShare of the batch's pruned-row updates (below that, the
    // merge-capable kernel's extra scalar state costs more than it saves)
    bool trsm_merge = false;
    // select_iters: per subdomain applied with the factor (not assembled),
    // and the prediction behind the choice
    std::vector<uint8_t> implicit_sub;
    std::vector<Prediction> pred;
    int32_t n_implicit = 0;
    hipGraphExec_t graph_exec = nullptr;        // captured assembly (use_graph)
    hipGraphExec_t impl_graph = nullptr;        // captured triangular sweeps of the implicit apply (use_graph)
    bool impl_ready = false;                    // implicit apply schedule and workspace built
    double trsm_u = 0, syrk_u = 0, trsm_d = 0, syrk_d = 0, trsm_r = 0, syrk_r = 0;
    // kernel timing: event pairs per kernel, pending until read
    bool timing = false;
    struct PendingTiming { int kernel; hipEvent_t a, b; };
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> event_pool;
    double ms_sum[kNumTimed] = {};
    int64_t ms_count[kNumTimed] = {};

    bool overlapped() const { return opt.assembly_kernels == 1; }
    // Overlapped assembly: TRSM of group g+1 on `st` runs while SYRK of group g
    // runs on the second stream (which waits for TRSM g through an event);
    // `st` finally waits for the last SYRK.  The two kernels keep their own
    // register and LDS budgets, so a CU can hold workgroups of both.
    hipError_t prepare_overlap() {           // at plan creation (not inside a graph capture)
        hipError_t e = hipSuccess;
        if (!aux && (e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking)) != hipSuccess) return e;
        while (ov_events.size() < g_tcnt.size() + 1) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
            ov_events.push_back(ev);
        }
        return hipSuccess;
    }
    hipError_t launch_overlapped(hipStream_t st) {
        hipError_t e = hipSuccess;
        const size_t ng = g_tcnt.size();
        if (!aux || ov_events.size() < ng + 1) return hipErrorNotReady;
        const DevTables t = tables();
        for (size_t g = 0; g < ng; ++g) {
            if ((e = launch_trsm(t, d_tile_order_g.p + g_toff[g], g_tcnt[g], st)) != hipSuccess) return e;
            if ((e = hipEventRecord(ov_events[g], st)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(aux, ov_events[g], 0)) != hipSuccess) return e;
            if ((e = launch_syrk(t, d_syrk_g.p + g_soff[g], g_stile[g], g_sblock[g], aux)) != hipSuccess) return e;
        }
        if ((e = hipEventRecord(ov_events[ng], aux)) != hipSuccess) return e;
        return hipStreamWaitEvent(st, ov_events[ng], 0);
    }
    // temporary-memory waves: TRSM then SYRK of each group in turn on `st`
    // (the next wave's TRSM overwrites X only after this wave's SYRK)
    hipError_t launch_waves(hipStream_t st) {
        hipError_t e = hipSuccess;
        const DevTables t = tables();
        for (size_t g = 0; g < g_tcnt.size(); ++g) {
            if ((e = launch_trsm(t, d_tile_order_g.p + g_toff[g], g_tcnt[g], st)) != hipSuccess) return e;
            if ((e = launch_syrk(t, d_syrk_g.p + g_soff[g], g_stile[g], g_sblock[g], st)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t launch_assembly(hipStream_t st, hipEvent_t* ev) {
        if (arena_elems > 0) {
            hipError_t e = hipSuccess;
            if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
            if ((e = launch_waves(st)) != hipSuccess) return e;
            if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
            return hipSuccess;
        }
        if (!overlapped()) return launch_assemble(tables(), st, ev);
        hipError_t e = hipSuccess;
        if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
        if ((e = launch_overlapped(st)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
        return hipSuccess;
    }
    hipError_t take_events(int k, hipEvent_t* out) {
        for (int i = 0; i < k; ++i) {
            if (event_pool.empty()) {
                hipEvent_t e;
                hipError_t err = hipEventCreate(&e);
                if (err != hipSuccess) return err;
                event_pool.push_back(e);
            }
            out[i] = event_pool.back();
            event_pool.pop_back();
        }
        return hipSuccess;
    }
    hipError_t drain_timing(bool wait) {
        std::vector<PendingTiming> keep;
        for (auto& p : pending) {
            if (!wait && hipEventQuery(p.b) != hipSuccess) { keep.push_back(p); continue; }
            hipError_t e = hipEventSynchronize(p.b);
            if (e != hipSuccess) return e;
            float ms = 0;
            e = hipEventElapsedTime(&ms, p.a, p.b);
            if (e != hipSuccess) return e;
            ms_sum[p.kernel] += ms;
            ms_count[p.kernel] += 1;
            event_pool.push_back(p.a);
            event_pool.push_back(p.b);
        }
        pending.swap(keep);
        return hipSuccess;
    }

    int64_t device_bytes() const {
        return (int64_t)(d_subs.count * sizeof(SubDev) + d_tiles.count * sizeof(TileDev) +
                         d_blocks.count * sizeof(BlockDev) + d_syrk.count * sizeof(SyrkItem) +
                         d_ftiles.count * sizeof(SyrkItem) + d_frows.count * sizeof(int2) +
                         d_part.count * 8 + d_tile_order.count * 4 +
                         d_tile_order_g.count * 4 + d_syrk_g.count * sizeof(SyrkItem) +
                         (d_rows.count + d_piv.count + d_pi.count + d_visit.count + d_ksteps.count) * 4 + d_vrows.count * 8 + d_sgn.count +
                         (d_lval.count + d_X.count + d_F.count) * 8 +
                         (d_lval32.count + d_X32.count + d_F32.count) * 4 +
                         (d_xwork.count + d_ywork.count + d_xoff.count) * 8 + (d_ifw.count + d_ibw.count) * sizeof(int2) +
                         (d_rptr.count + d_rpos.count) * 4 + (d_rptr_off.count + d_ubuf.count) * 8 +
                         (d_ifw_h.count + d_ibw_h.count) * sizeof(int2) + d_impl_list.count * 4);
    }
    void release() {
        d_subs.release(); d_tiles.release(); d_blocks.release(); d_syrk.release();
        d_ftiles.release(); d_frows.release(); d_part.release();
        d_tile_order.release(); d_tile_order_g.release(); d_syrk_g.release();
        d_rows.release(); d_piv.release(); d_pi.release(); d_visit.release(); d_ksteps.release(); d_vrows.release(); d_sgn.release();
        d_lval.release(); d_X.release(); d_F.release();
        d_lval32.release(); d_X32.release(); d_F32.release();
        d_xwork.release(); d_ywork.release(); d_xoff.release();
        d_ifw.release(); d_ibw.release(); d_rptr_off.release(); d_rptr.release(); d_rpos.release(); d_ubuf.release();
        d_ifw_h.release(); d_ibw_h.release(); d_impl_list.release();
        if (h_lval) (void)hipHostFree(h_lval);
        h_lval = nullptr;
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
        if (impl_graph) (void)hipGraphExecDestroy(impl_graph);
        impl_graph = nullptr;
        for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (auto& e : event_pool) (void)hipEventDestroy(e);
        pending.clear();
        event_pool.clear();
        for (auto& e : ov_events) (void)hipEventDestroy(e);
        ov_events.clear();
        if (aux) (void)hipStreamDestroy(aux);
        aux = nullptr;
    }
    DevTables tables() const {
        DevTables t;
        t.subs = d_subs.p; t.tiles = d_tiles.p; t.blocks = d_blocks.p; t.rows = d_rows.p; t.visit = d_visit.p;
        t.ksteps = d_ksteps.p;
        t.vrows = d_vrows.p;
        t.lval = d_lval.p; t.piv = d_piv.p; t.pi = d_pi.p; t.sgn = d_sgn.p; t.syrk = d_syrk.p;
        t.X = d_X.p; t.F = d_F.p;
        t.lval32 = d_lval32.p; t.X32 = d_X32.p; t.F32 = d_F32.p;
        t.ftiles = d_ftiles.p;
        t.frows = d_frows.p;
        t.part = d_part.p;
        t.tile_order = d_tile_order.p;
        t.trsm_merge = trsm_merge;
        t.ntiles = (int64_t)h_tile_order.size();
        t.nsyrk = (int64_t)h_syrk.size();
        t.nsyrk_tile = nsyrk_tile;
        t.nftiles = (int64_t)h_ftiles.size();
        t.nfrows = (int64_t)h_frows.size();
        return t;
    }
};

namespace {

// Mean ms per sc_assemble of a temporary plan of `ns` subdomains with
// options `o` (one warm-up call, then `reps` timed calls between events).
sc_status_t time_candidate(const sc_subdomain_desc_t* sub, int32_t ns, const sc_options_t& o,
                           const double* const* vals, int32_t reps, void* stream, hipEvent_t e0, hipEvent_t e1,
                           double* ms_out) {
    hipStream_t st = (hipStream_t)stream;
    sc_plan_t P = nullptr;
    sc_status_t status = sc_plan_create(sub, ns, &o, stream, &P);
    if (status == SC_OK) status = sc_factor(P, vals, stream, nullptr, nullptr);
    if (status == SC_OK) status = sc_assemble(P, stream);
    float ms = 0.f;
    if (status == SC_OK) {
        hipError_t e = hipEventRecord(e0, st);
        for (int32_t r = 0; r < reps && e == hipSuccess; ++r)
            if (sc_assemble(P, stream) != SC_OK) e = hipErrorUnknown;
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) status = fail(SC_ERR_DEVICE, "autotune timing failed");
    }
    const std::string keep = g_last_error;
    sc_plan_destroy(P);
    g_last_error = keep;
    *ms_out = ms / reps;
    return status;
}

std::string device_key() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string k = std::string(prop.gcnArchName) + "|" + prop.name;
    for (char& c : k)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    return k;
}

}  // namespace

extern "C" {

const char* sc_last_error(void) { return g_last_error.c_str(); }

sc_status_t sc_plan_create(const sc_subdomain_desc_t* sd, int32_t nsub, const sc_options_t* opt,
                           void* stream, sc_plan_t* out) {
    g_last_error.clear();
    if (!out) return fail(SC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nsub < 0 || (nsub > 0 && !sd)) return fail(SC_ERR_INVALID_ARG, "bad subdomain array");
    std::unique_ptr<sc_plan_s> P(new (std::nothrow) sc_plan_s());
    if (!P) return fail(SC_ERR_OOM, "host allocation failed");
    if (opt) P->opt = *opt;
    PlanOptions& po = P->popt;
    {
        const std::string err = to_plan_options(P->opt, po);
        if (!err.empty()) return fail(SC_ERR_INVALID_ARG, err);
    }
    P->mixed = P->opt.precision == SC_PREC_MIXED;
    if (P->opt.arena_cap_bytes > 0) {
        if (P->opt.assembly_kernels == 1)
            return fail(SC_ERR_UNSUPPORTED, "arena_cap_bytes with assembly_kernels = 1: the waves run one after "
                                            "the other on one X buffer and cannot overlap");
        P->arena_elems = std::max<int64_t>(1, P->opt.arena_cap_bytes / (P->mixed ? 4 : 8));
    }
    P->nsub = nsub;
    P->plans.resize(nsub);
    P->kval_count.resize(nsub);
    std::vector<std::string> errs(nsub);
    std::vector<int> codes(nsub, 0);
    const int nthr = P->opt.n_threads > 0 ? P->opt.n_threads : omp_get_max_threads();
    // per-subdomain settings from the autotuner's size classes
    P->syrk_kind.assign(nsub, P->opt.syrk_kind);
    std::vector<PlanOptions> spo(nsub, po);
    for (int32_t i = 0; i < nsub; ++i)
        for (int32_t c = 0; c < P->opt.ntune_classes; ++c) {
            const sc_tune_class_t& k = P->opt.tune_classes[c];
            if (sd[i].n < k.n_lo || sd[i].n >= k.n_hi) continue;
            if (k.panel_width) spo[i].panel_width = k.panel_width;
            if (k.block_split >= 0) spo[i].block_split = k.block_split;
            P->syrk_kind[i] = k.syrk_kind;
            break;
        }
    P->opt.tune_classes = nullptr;          // borrowed for this call only
    P->opt.ntune_classes = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int32_t i = 0; i < nsub; ++i) {
        try {
            errs[i] = plan_subdomain(sd[i], spo[i], P->opt.lower_only_csr != 0, P->plans[i], codes[i]);
        } catch (const std::bad_alloc&) {
            errs[i] = "host allocation failed";
            codes[i] = 3;
        } catch (...) {
            errs[i] = "planner failed";
            codes[i] = 1;
        }
        if (errs[i].empty() && sd[i].n > 0) P->kval_count[i] = sd[i].kreg_rowptr[sd[i].n];
    }
    for (int32_t i = 0; i < nsub; ++i)
        if (!errs[i].empty())
            return fail(codes[i] == 3 ? SC_ERR_OOM : SC_ERR_INVALID_ARG,
                        "subdomain " + std::to_string(i) + ": " + errs[i]);

    // ---- tables
    // SYRK items per subdomain: 128 x 128 tiles (large subdomains) or 64 x 64
    // blocks
    std::vector<std::vector<SyrkItem>> sub_tiles(nsub), sub_blocks(nsub);
    std::vector<int64_t> x_elems(nsub, 0);      // X slab elements of each subdomain
    int64_t blk = 0, rows = 0, lv = 0, colo = 0, xo = 0, fo = 0, dual = 0;
    int64_t upd_rows = 0, merged_rows = 0;      // TRSM pruned-row updates, and those the merged pairs save
    P->implicit_sub.assign(nsub, 0);
    P->pred.resize(nsub);
    for (int32_t i = 0; i < nsub; ++i) {
        P->pred[i] = predict(P->plans[i], P->mixed, P->opt);
        if (P->opt.select_iters > 0 && P->pred[i].n_star > (double)P->opt.select_iters) {
            P->implicit_sub[i] = 1;
            ++P->n_implicit;
        }
    }
    for (int32_t i = 0; i < nsub; ++i) {
        const SubPlan& sp = P->plans[i];
        const bool impl = P->implicit_sub[i] != 0;
        SubDev s{};
        s.n = sp.n;
        s.m = sp.m;
        s.nblocks = (int32_t)sp.blocks.size();
        s.ntiles = (sp.m + kTile - 1) / kTile;
        s.blk_off = blk;
        s.rows_off = rows;
        s.lval_off = lv;
        s.col_off = colo;
        s.tile_off = (int64_t)P->h_tiles.size();
        s.F_off = fo;
        s.dual_off = dual;
        {
            // merged pairs of the TRSM's updates below (unless disabled), and
            // the pruned-row updates of the tiles' visits they save
            const std::vector<int32_t> pair =
                P->opt.disable_pair_merge ? std::vector<int32_t>(sp.blocks.size(), 0) : merge_pairs(sp);
            for (size_t k = 0; k < sp.blocks.size(); ++k) {
                const BlockDesc& b = sp.blocks[k];
                P->h_blocks.push_back(
                    BlockDev{b.row0, b.w, b.nbelow, pair[k], b.lval_off, b.rows_off, b.aoff, b.linv_off});
            }
            if (!impl)
                for (int32_t t = 0; t + 1 < (int32_t)sp.visit_ptr.size(); ++t)
                    for (int64_t k = sp.visit_ptr[t]; k < sp.visit_ptr[t + 1]; ++k) {
                        const int32_t b = sp.visit[k];
                        upd_rows += sp.blocks[b].nbelow;
                        if (pair[b] && k + 1 < sp.visit_ptr[t + 1] && sp.visit[k + 1] == b + 1)
                            merged_rows += sp.blocks[b + 1].nbelow;
                    }
        }
        for (int32_t t = 0; t < s.ntiles; ++t) {
            TileDev T{};
            T.sub = i;
            T.tile = t;
            T.ncols = std::min(kTile, sp.m - t * kTile);
            T.kstart = po.staircase ? sp.piv[(size_t)t * kTile] : 0;
            T.x_off = xo;
            xo += (int64_t)(sp.n - T.kstart) * kTile;
            x_elems[i] += (int64_t)(sp.n - T.kstart) * kTile;
            for (int w = 0; w < 4; ++w) {
                const int c = t * kTile + w * kStripe;
                if (w * kStripe >= T.ncols) T.start_block[w] = s.nblocks;
                else T.start_block[w] = po.staircase ? sp.block_of_row[sp.piv[c]] : 0;
            }
            T.visit_off = (int64_t)P->h_visit.size();
            T.nvisit = (int32_t)(sp.visit_ptr[t + 1] - sp.visit_ptr[t]);
            P->h_visit.insert(P->h_visit.end(), sp.visit.begin() + sp.visit_ptr[t], sp.visit.begin() + sp.visit_ptr[t + 1]);
            P->h_vrows.insert(P->h_vrows.end(), sp.visit_rows.begin() + sp.visit_ptr[t],
                              sp.visit_rows.begin() + sp.visit_ptr[t + 1]);
            P->h_tiles.push_back(T);
        }
        const int32_t nst = (sp.m + kSyrkTile - 1) / kSyrkTile;
        s.ftile_off = (int64_t)P->h_ftiles.size();
        for (int32_t I = 0; I < nst && !impl; ++I) {     // implicit subdomains: no F
            P->h_frows.push_back(make_int2(i, I));
            for (int32_t J = 0; J <= I; ++J) P->h_ftiles.push_back(SyrkItem{i, I, J, 0, 0});
        }
        {
            // SYRK items with their 16-row steps where both sides can hold
            // nonzero X rows; items without any are structurally zero and are
            // left to the one-time clear of F
            const int32_t nw = sp.mask_words;
            auto mask = [&](int32_t t64, int32_t q) -> uint64_t {
                return t64 < s.ntiles ? sp.step_mask[(size_t)t64 * nw + q] : 0;
            };
            const bool blocks = P->syrk_kind[i] == 1 ||
                                (P->syrk_kind[i] == 0 && sp.n <= (P->mixed ? kSyrkBlockMaxNMixed : kSyrkBlockMaxN));
            if (blocks) {
                for (int32_t I = 0; I < s.ntiles; ++I)
                    for (int32_t J = 0; J <= I; ++J) {
                        SyrkItem it{i, I, J, 0, (int64_t)P->h_ksteps.size()};
                        for (int32_t q = 0; q < nw; ++q) {
                            uint64_t b = mask(I, q) & mask(J, q);
                            while (b) {
                                P->h_ksteps.push_back(16 * (64 * q + __builtin_ctzll(b)));
                                b &= b - 1;
                            }
                        }
                        it.nsteps = (int32_t)(P->h_ksteps.size() - it.step_off);
                        if (it.nsteps > 0 && !impl) sub_blocks[i].push_back(it);
                    }
            } else {
                for (int32_t I = 0; I < nst; ++I)
                    for (int32_t J = 0; J <= I; ++J) {
                        SyrkItem it{i, I, J, 0, (int64_t)P->h_ksteps.size()};
                        for (int32_t q = 0; q < nw; ++q) {
                            const uint64_t m0 = mask(2 * I, q), m1 = mask(2 * I + 1, q);
                            const uint64_t m2 = mask(2 * J, q), m3 = mask(2 * J + 1, q);
                            uint64_t b = (m0 | m1) & (m2 | m3);
                            while (b) {
                                const int bit = __builtin_ctzll(b);
                                const int32_t tag = (int32_t)(((m0 >> bit) & 1) | (((m1 >> bit) & 1) << 1) |
                                                              (((m2 >> bit) & 1) << 2) | (((m3 >> bit) & 1) << 3));
                                P->h_ksteps.push_back(16 * (64 * q + bit) | tag << kStepSlabShift);
                                b &= b - 1;
                            }
                        }
                        it.nsteps = (int32_t)(P->h_ksteps.size() - it.step_off);
                        if (it.nsteps > 0 && !impl) sub_tiles[i].push_back(it);
                    }
            }
        }
        blk += s.nblocks;
        rows += ((int64_t)sp.brows.size() + 3) / 4 * 4;
        lv += sp.bval;
        colo += sp.m;
        fo += (int64_t)nst * (nst + 1) / 2 * kFTileElems;   // packed lower tiles
        dual += sp.m;
        P->h_subs.push_back(s);
        P->trsm_u += sp.trsm_useful;
        P->syrk_u += sp.syrk_useful;
        P->trsm_d += sp.trsm_dense;
        P->syrk_d += sp.syrk_dense;
        P->trsm_r += sp.trsm_reach;
        P->syrk_r += sp.syrk_reach;
    }
    if (P->arena_elems > 0)
        for (int32_t i = 0; i < nsub; ++i)
            if (x_elems[i] > P->arena_elems)
                return fail(SC_ERR_OOM, "arena_cap_bytes = " + std::to_string(P->opt.arena_cap_bytes) +
                                            " is below the X slabs of subdomain " + std::to_string(i) + " (" +
                                            std::to_string(x_elems[i] * (P->mixed ? 4 : 8)) + " bytes)");
    // ---- XCD-aware work lists: subdomains go to XCDs by longest-processing-
    // time on their useful flops; XCD x receives workgroups x, x + 8, ...
    {
        std::vector<int32_t> byc(nsub);
        std::iota(byc.begin(), byc.end(), 0);
        std::stable_sort(byc.begin(), byc.end(), [&](int32_t a, int32_t b) {
            return P->plans[a].trsm_useful + P->plans[a].syrk_useful >
                   P->plans[b].trsm_useful + P->plans[b].syrk_useful;
        });
        std::vector<double> load(kNumXcd, 0.0);
        std::vector<std::vector<int32_t>> xsub(kNumXcd);
        for (int32_t i : byc) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[x] += P->plans[i].trsm_useful + P->plans[i].syrk_useful + 1.0;
            xsub[x].push_back(i);
        }
        // SYRK list of a set of subdomains per XCD: the 128 x 128 tiles, then
        // the 64 x 64 blocks, each part interleaved over the XCDs
        auto syrk_list = [&](const std::vector<std::vector<int32_t>>& subs_of_xcd, std::vector<SyrkItem>& out,
                             int64_t& ntile, int64_t& nblock) {
            for (int part = 0; part < 2; ++part) {
                const auto& src = part == 0 ? sub_tiles : sub_blocks;
                std::vector<std::vector<SyrkItem>> xl(kNumXcd);
                size_t len = 0;
                for (int x = 0; x < kNumXcd; ++x) {
                    for (int32_t i : subs_of_xcd[x]) xl[x].insert(xl[x].end(), src[i].begin(), src[i].end());
                    len = std::max(len, xl[x].size());
                }
                const size_t base = out.size();
                out.resize(base + len * kNumXcd, SyrkItem{-1, 0, 0, 0, 0});
                for (int x = 0; x < kNumXcd; ++x)
                    for (size_t k = 0; k < xl[x].size(); ++k) out[base + k * kNumXcd + x] = xl[x][k];
                (part == 0 ? ntile : nblock) = (int64_t)(len * kNumXcd);
            }
        };
        // the tiles of one subdomain in order of decreasing visit count, its
        // SYRK items in order of decreasing step count (long items first)
        auto push_tiles = [&](std::vector<int32_t>& list, int32_t i) {
            if (P->implicit_sub[i]) return;           // applied with the factor: no tiles
            const SubDev& sd = P->h_subs[i];
            const size_t b0 = list.size();
            for (int32_t t = 0; t < sd.ntiles; ++t) list.push_back((int32_t)(sd.tile_off + t));
            std::stable_sort(list.begin() + b0, list.end(), [&](int32_t a, int32_t b) {
                return P->h_tiles[a].nvisit > P->h_tiles[b].nvisit;
            });
        };
        auto by_steps = [](const SyrkItem& a, const SyrkItem& b) { return a.nsteps > b.nsteps; };
        for (int32_t i = 0; i < nsub; ++i) {
            std::stable_sort(sub_tiles[i].begin(), sub_tiles[i].end(), by_steps);
            std::stable_sort(sub_blocks[i].begin(), sub_blocks[i].end(), by_steps);
        }
        std::vector<std::vector<int32_t>> xt(kNumXcd);
        // groups for the overlapped assembly
        // groups of subdomains: without an arena cap every XCD's list cut in
        // kOverlapGroups consecutive parts (overlapped assembly, pipelined
        // preprocessing); with a cap (temporary-memory waves) the subdomains
        // in XCD-interleaved order (largest first) packed greedily into waves
        // whose X slabs fit the cap, each wave's slabs at the same offsets
        std::vector<std::vector<int32_t>> groups;
        std::vector<int32_t> xcd_of(nsub, 0);
        for (int x = 0; x < kNumXcd; ++x)
            for (int32_t i : xsub[x]) xcd_of[i] = x;
        {
            size_t lmax = 0;
            for (int x = 0; x < kNumXcd; ++x) lmax = std::max(lmax, xsub[x].size());
            if (P->arena_elems > 0) {
                groups.emplace_back();
                int64_t cur = 0;
                for (size_t k = 0; k < lmax; ++k)
                    for (int x = 0; x < kNumXcd; ++x) {
                        if (k >= xsub[x].size()) continue;
                        const int32_t i = xsub[x][k];
                        if (!groups.back().empty() && cur + x_elems[i] > P->arena_elems) {
                            groups.emplace_back();
                            cur = 0;
                        }
                        groups.back().push_back(i);
                        cur += x_elems[i];
                    }
            } else {
                const int ng = (int)std::max<size_t>(1, std::min<size_t>(kOverlapGroups, lmax));
                for (int gi = 0; gi < ng; ++gi) {
                    groups.emplace_back();
                    for (int x = 0; x < kNumXcd; ++x) {
                        const size_t L = xsub[x].size();
                        for (size_t k = L * gi / ng; k < L * (gi + 1) / ng; ++k) groups.back().push_back(xsub[x][k]);
                    }
                }
            }
            for (const std::vector<int32_t>& grp : groups) {
                std::vector<std::vector<int32_t>> gt(kNumXcd), gsub(kNumXcd);
                for (int32_t i : grp) gsub[xcd_of[i]].push_back(i);
                size_t lt = 0;
                for (int x = 0; x < kNumXcd; ++x) {
                    for (int32_t i : gsub[x]) push_tiles(gt[x], i);
                    lt = std::max(lt, gt[x].size());
                }
                P->g_sub_off.push_back((int64_t)P->g_sub.size());
                {
                    size_t lg = 0;
                    for (int x = 0; x < kNumXcd; ++x) lg = std::max(lg, gsub[x].size());
                    for (size_t k = 0; k < lg; ++k)       // largest subdomains first
                        for (int x = 0; x < kNumXcd; ++x)
                            if (k < gsub[x].size()) P->g_sub.push_back(gsub[x][k]);
                }
                P->g_toff.push_back((int64_t)P->h_tile_order_g.size());
                P->g_tcnt.push_back((int64_t)(lt * kNumXcd));
                P->g_soff.push_back((int64_t)P->h_syrk_g.size());
                int64_t nt = 0, nb = 0;
                syrk_list(gsub, P->h_syrk_g, nt, nb);
                P->g_stile.push_back(nt);
                P->g_sblock.push_back(nb);
                P->h_tile_order_g.resize(P->h_tile_order_g.size() + lt * kNumXcd, -1);
                for (int x = 0; x < kNumXcd; ++x)
                    for (size_t k = 0; k < gt[x].size(); ++k)
                        P->h_tile_order_g[P->g_toff.back() + (int64_t)(k * kNumXcd + x)] = gt[x][k];
            }
        }
        P->g_sub_off.push_back((int64_t)P->g_sub.size());
        // factor values group after group, so that each group's upload is one copy
        {
            int64_t off = 0;
            for (size_t g = 0; g + 1 < P->g_sub_off.size(); ++g) {
                P->g_lval.push_back(off);
                for (int64_t k = P->g_sub_off[g]; k < P->g_sub_off[g + 1]; ++k) {
                    const int32_t i = P->g_sub[k];
                    P->h_subs[i].lval_off = off;
                    off += P->plans[i].bval;
                }
            }
            P->g_lval.push_back(off);
            if (off != lv || (int64_t)P->g_sub.size() != nsub)
                return fail(SC_ERR_INVALID_ARG, "internal: subdomain groups do not cover the batch");
        }
        if (P->arena_elems > 0) {
            // temporary-memory waves: the X slabs of each wave start at 0
            xo = 0;
            for (const std::vector<int32_t>& grp : groups) {
                int64_t off = 0;
                for (int32_t i : grp) {
                    const SubDev& sd = P->h_subs[i];
                    for (int32_t t = 0; t < sd.ntiles; ++t) {
                        TileDev& T = P->h_tiles[sd.tile_off + t];
                        T.x_off = off;
                        off += (int64_t)(sd.n - T.kstart) * kTile;
                    }
                }
                xo = std::max(xo, off);
            }
        }
        for (int x = 0; x < kNumXcd; ++x)
            for (int32_t i : xsub[x]) push_tiles(xt[x], i);
        size_t lt = 0;
        for (int x = 0; x < kNumXcd; ++x) lt = std::max(lt, xt[x].size());
        P->h_tile_order.assign(lt * kNumXcd, -1);
        for (int x = 0; x < kNumXcd; ++x)
            for (size_t k = 0; k < xt[x].size(); ++k) P->h_tile_order[k * kNumXcd + x] = xt[x][k];
        P->h_syrk.clear();
        int64_t nb = 0;
        syrk_list(xsub, P->h_syrk, P->nsyrk_tile, nb);
    }
    P->nval_total = lv;
    P->trsm_merge = merged_rows > 0 && (double)merged_rows >= kMergeMinShare * (double)upd_rows;
    rows += 64;                            // the TRSM reads whole 64-entry groups of a row list
    P->nrows_total = rows;
    P->ncol_total = colo;
    P->X_total = xo;
    P->F_total = fo;
    P->dual_total = dual;
    {
        // chunks of the allocation-free apply: consecutive whole subdomains
        ApplyChunk cur{0, 0, 0, 0};
        for (int32_t i = 0; i < nsub; ++i) {
            const int64_t nst = P->implicit_sub[i] ? 0 : ((int64_t)P->h_subs[i].m + kSyrkTile - 1) / kSyrkTile;
            const int64_t nt = nst * (nst + 1) / 2;
            if (nt > kApplyScratchTiles) {
                if (P->noalloc_too_big < 0) P->noalloc_too_big = i;
            } else if (cur.t1 - cur.t0 + nt > kApplyScratchTiles) {
                P->h_chunks.push_back(cur);
                cur = ApplyChunk{cur.t1, cur.t1, cur.r1, cur.r1};
            }
            cur.t1 += nt;
            cur.r1 += nst;
        }
        if (cur.t1 > cur.t0) P->h_chunks.push_back(cur);
    }

    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipGetDevice(&P->device));
    // device address of the fixed scratch array of the allocation-free apply
    // (looked up once per device; an error is reported by that entry point)
    P->scratch_err = apply_scratch_init(P->device, &P->scratch);
    sc_plan_s* p = P.get();
    auto cleanup_fail = [&](sc_status_t s, const std::string& m) { p->release(); return fail(s, m); };
#define ALLOC(buf, n)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (buf).alloc(n);                                                      \
        if (e_ != hipSuccess)                                                                \
            return cleanup_fail(e_ == hipErrorOutOfMemory ? SC_ERR_OOM : SC_ERR_DEVICE,      \
                                std::string("hipMalloc ") + #buf + ": " + hipGetErrorString(e_)); \
    } while (0)
    ALLOC(p->d_subs, p->h_subs.size());
    ALLOC(p->d_tiles, p->h_tiles.size());
    ALLOC(p->d_blocks, p->h_blocks.size());
    ALLOC(p->d_syrk, p->h_syrk.size());
    ALLOC(p->d_ftiles, p->h_ftiles.size());
    ALLOC(p->d_frows, p->h_frows.size());
    ALLOC(p->d_part, p->h_ftiles.size() * 256);
    ALLOC(p->d_tile_order, p->h_tile_order.size());
    ALLOC(p->d_tile_order_g, p->h_tile_order_g.size());
    ALLOC(p->d_syrk_g, p->h_syrk_g.size());
    ALLOC(p->d_rows, (size_t)rows);
    ALLOC(p->d_visit, std::max<size_t>(1, p->h_visit.size()));
    ALLOC(p->d_ksteps, std::max<size_t>(1, p->h_ksteps.size()));
    ALLOC(p->d_vrows, std::max<size_t>(1, p->h_vrows.size()));
    ALLOC(p->d_piv, (size_t)colo);
    ALLOC(p->d_pi, (size_t)colo);
    ALLOC(p->d_sgn, (size_t)colo);
    ALLOC(p->d_lval, (size_t)lv);
    if (p->mixed) {
        ALLOC(p->d_lval32, (size_t)lv);
        ALLOC(p->d_X32, (size_t)xo);
        ALLOC(p->d_F32, (size_t)fo);
    } else {
        ALLOC(p->d_X, (size_t)xo);
        ALLOC(p->d_F, (size_t)fo);
    }
#undef ALLOC
    {
        hipError_t e = hipHostMalloc((void**)&p->h_lval, std::max<size_t>(1, (size_t)lv) * sizeof(double),
                                     hipHostMallocDefault);
        if (e != hipSuccess) return cleanup_fail(SC_ERR_OOM, "pinned host allocation failed");
    }
    // flatten per-subdomain arrays
    std::vector<int32_t> h_rows((size_t)rows, -1), h_piv((size_t)colo), h_pi((size_t)colo);
    std::vector<int8_t> h_sgn((size_t)colo);
    for (int32_t i = 0; i < nsub; ++i) {
        const SubPlan& sp = P->plans[i];
        const SubDev& s = P->h_subs[i];
        std::copy(sp.brows.begin(), sp.brows.end(), h_rows.begin() + s.rows_off);
        std::copy(sp.piv.begin(), sp.piv.end(), h_piv.begin() + s.col_off);
        std::copy(sp.pi.begin(), sp.pi.end(), h_pi.begin() + s.col_off);
        std::copy(sp.sign_sorted.begin(), sp.sign_sorted.end(), h_sgn.begin() + s.col_off);
    }
    auto up = [&](void* d, const void* h, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(p->d_subs.p, p->h_subs.data(), p->h_subs.size() * sizeof(SubDev));
    if (e == hipSuccess) e = up(p->d_tiles.p, p->h_tiles.data(), p->h_tiles.size() * sizeof(TileDev));
    if (e == hipSuccess) e = up(p->d_blocks.p, p->h_blocks.data(), p->h_blocks.size() * sizeof(BlockDev));
    if (e == hipSuccess) e = up(p->d_syrk.p, p->h_syrk.data(), p->h_syrk.size() * sizeof(SyrkItem));
    if (e == hipSuccess) e = up(p->d_ftiles.p, p->h_ftiles.data(), p->h_ftiles.size() * sizeof(SyrkItem));
    if (e == hipSuccess) e = up(p->d_frows.p, p->h_frows.data(), p->h_frows.size() * sizeof(int2));
    if (e == hipSuccess) e = up(p->d_tile_order.p, p->h_tile_order.data(), p->h_tile_order.size() * 4);
    if (e == hipSuccess) e = up(p->d_tile_order_g.p, p->h_tile_order_g.data(), p->h_tile_order_g.size() * 4);
    if (e == hipSuccess) e = up(p->d_syrk_g.p, p->h_syrk_g.data(), p->h_syrk_g.size() * sizeof(SyrkItem));
    if (e == hipSuccess && p->overlapped()) e = p->prepare_overlap();
    if (e == hipSuccess) e = up(p->d_rows.p, h_rows.data(), h_rows.size() * 4);
    if (e == hipSuccess) e = up(p->d_visit.p, p->h_visit.data(), p->h_visit.size() * 4);
    if (e == hipSuccess) e = up(p->d_ksteps.p, p->h_ksteps.data(), p->h_ksteps.size() * 4);
    if (e == hipSuccess) e = up(p->d_vrows.p, p->h_vrows.data(), p->h_vrows.size() * 8);
    // F is cleared once: the SYRK never writes its structurally zero blocks
    // nor the columns past m of the last tiles
    if (e == hipSuccess && fo > 0)
        e = p->mixed ? hipMemsetAsync(p->d_F32.p, 0, (size_t)fo * sizeof(float), st)
                     : hipMemsetAsync(p->d_F.p, 0, (size_t)fo * sizeof(double), st);
    if (e == hipSuccess) e = up(p->d_piv.p, h_piv.data(), h_piv.size() * 4);
    if (e == hipSuccess) e = up(p->d_pi.p, h_pi.data(), h_pi.size() * 4);
    if (e == hipSuccess) e = up(p->d_sgn.p, h_sgn.data(), h_sgn.size());
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // host vectors go out of scope
    if (e != hipSuccess) return cleanup_fail(SC_ERR_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
    *out = P.release();
    return SC_OK;
}

sc_status_t sc_factor(sc_plan_t P, const double* const* kreg_vals, void* stream, int32_t* failed_sub,
                      int32_t* failed_col) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (P->nsub > 0 && !kreg_vals) return fail(SC_ERR_INVALID_ARG, "kreg_vals is NULL");
    for (int32_t i = 0; i < P->nsub; ++i)
        if (!kreg_vals[i] && P->kval_count[i] > 0)
            return fail(SC_ERR_INVALID_ARG, "kreg_vals[" + std::to_string(i) + "] is NULL");
    HIP_TRY(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    // the previous upload may still read h_lval
    HIP_TRY(hipStreamSynchronize(st));
    P->factored = false;
    P->assembled = false;
    std::vector<int64_t> bad(P->nsub, -1);
    const int nthr = P->opt.n_threads > 0 ? P->opt.n_threads : omp_get_max_threads();
    bool oom = false;
#pragma omp parallel num_threads(nthr)
    {
        std::vector<double> sn;     // supernodal values of the subdomain being factored
#pragma omp for schedule(dynamic, 1)
        for (int32_t i = 0; i < P->nsub; ++i) {
            const SubPlan& sp = P->plans[i];
            try {
                sn.resize((size_t)std::max<int64_t>(1, sp.nval));
            } catch (const std::bad_alloc&) {
#pragma omp atomic write
                oom = true;
                continue;
            }
            bad[i] = factor_numeric(sp, kreg_vals[i], sn.data());
            if (bad[i] < 0) repack_blocks(sp, sn.data(), P->h_lval + P->h_subs[i].lval_off);
        }
    }
    if (oom) return fail(SC_ERR_OOM, "host allocation failed in sc_factor");
    for (int32_t i = 0; i < P->nsub; ++i)
        if (bad[i] >= 0) {
            if (failed_sub) *failed_sub = i;
            if (failed_col) *failed_col = (int32_t)bad[i];
            return fail(SC_ERR_NOT_SPD, "subdomain " + std::to_string(i) + ": pivot of permuted column " +
                                            std::to_string(bad[i]) + " is not positive");
        }
    if (P->nval_total > 0)
        HIP_TRY(hipMemcpyAsync(P->d_lval.p, P->h_lval, (size_t)P->nval_total * sizeof(double),
                               hipMemcpyHostToDevice, st));
    if (P->mixed) HIP_TRY(launch_convert_f32(P->d_lval.p, P->d_lval32.p, P->nval_total, st));
    P->factored = true;
    return SC_OK;
}

sc_status_t sc_preprocess(sc_plan_t P, const double* const* kreg_vals, void* stream, int32_t* failed_sub,
                          int32_t* failed_col) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (P->nsub > 0 && !kreg_vals) return fail(SC_ERR_INVALID_ARG, "kreg_vals is NULL");
    for (int32_t i = 0; i < P->nsub; ++i)
        if (!kreg_vals[i] && P->kval_count[i] > 0)
            return fail(SC_ERR_INVALID_ARG, "kreg_vals[" + std::to_string(i) + "] is NULL");
    HIP_TRY(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(st));   // an earlier upload may still read h_lval
    P->factored = false;
    P->assembled = false;
    const int64_t ng = (int64_t)P->g_sub_off.size() - 1;
    std::vector<int32_t> group_of(P->nsub, 0);
    std::vector<int64_t> left(ng, 0);
    for (int64_t g = 0; g < ng; ++g) {
        left[g] = P->g_sub_off[g + 1] - P->g_sub_off[g];
        for (int64_t k = P->g_sub_off[g]; k < P->g_sub_off[g + 1]; ++k) group_of[P->g_sub[k]] = (int32_t)g;
    }
    std::vector<int64_t> bad(P->nsub, -1);
    const DevTables t = P->tables();
    std::mutex mu;                       // guards left[], next and the launches
    int64_t next = 0;                    // first group not yet launched
    bool stop = false;                   // a pivot failed or a HIP call failed: launch nothing more
    hipError_t herr = hipSuccess;
    bool oom = false;
    // launches every consecutive group whose subdomains are all factored, in
    // group order, on `st`: its factor values (one copy), the FP32 copy in
    // mixed precision, its TRSM tiles and its SYRK items
    auto launch_ready = [&]() {
        while (!stop && next < ng && left[next] == 0) {
            const int64_t g = next++;
            const int64_t v0 = P->g_lval[g], nv = P->g_lval[g + 1] - v0;
            hipError_t e = hipSetDevice(P->device);
            if (e == hipSuccess && nv > 0)
                e = hipMemcpyAsync(P->d_lval.p + v0, P->h_lval + v0, (size_t)nv * sizeof(double),
                                   hipMemcpyHostToDevice, st);
            if (e == hipSuccess && P->mixed && nv > 0) e = launch_convert_f32(P->d_lval.p + v0, P->d_lval32.p + v0, nv, st);
            if (e == hipSuccess) e = launch_trsm(t, P->d_tile_order_g.p + P->g_toff[g], P->g_tcnt[g], st);
            if (e == hipSuccess) e = launch_syrk(t, P->d_syrk_g.p + P->g_soff[g], P->g_stile[g], P->g_sblock[g], st);
            if (e != hipSuccess) { herr = e; stop = true; }
        }
    };
    const int nthr = P->opt.n_threads > 0 ? P->opt.n_threads : omp_get_max_threads();
#pragma omp parallel num_threads(nthr)
    {
        std::vector<double> sn;
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < (int64_t)P->g_sub.size(); ++k) {
            const int32_t i = P->g_sub[k];
            const SubPlan& sp = P->plans[i];
            bool ok = true;
            try {
                sn.resize((size_t)std::max<int64_t>(1, sp.nval));
            } catch (const std::bad_alloc&) {
                ok = false;
            }
            if (ok) {
                bad[i] = factor_numeric(sp, kreg_vals[i], sn.data());
                if (bad[i] < 0) repack_blocks(sp, sn.data(), P->h_lval + P->h_subs[i].lval_off);
            }
            std::lock_guard<std::mutex> lk(mu);
            if (!ok) { oom = true; stop = true; }
            if (bad[i] >= 0) stop = true;
            --left[group_of[i]];
            launch_ready();
        }
    }
    if (oom) return fail(SC_ERR_OOM, "host allocation failed in sc_preprocess");
    for (int32_t i = 0; i < P->nsub; ++i)
        if (bad[i] >= 0) {
            if (failed_sub) *failed_sub = i;
            if (failed_col) *failed_col = (int32_t)bad[i];
            return fail(SC_ERR_NOT_SPD, "subdomain " + std::to_string(i) + ": pivot of permuted column " +
                                            std::to_string(bad[i]) + " is not positive");
        }
    if (herr != hipSuccess)
        return fail(herr == hipErrorOutOfMemory ? SC_ERR_OOM : SC_ERR_DEVICE,
                    std::string("sc_preprocess launch: ") + hipGetErrorString(herr));
    if (next != ng) return fail(SC_ERR_DEVICE, "sc_preprocess: not every group was launched");
    P->factored = true;
    P->assembled = true;
    return SC_OK;
}

sc_status_t sc_assemble(sc_plan_t P, void* stream) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (!P->factored) return fail(SC_ERR_STATE, "sc_assemble before sc_factor");
    HIP_TRY(hipSetDevice(P->device));
    if (P->opt.use_graph && !P->timing) {
        if (!P->graph_exec) {
            // capture on a private stream (the caller's may be the null stream,
            // which cannot be captured), replay on the caller's stream
            hipStream_t cap;
            HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t el = P->launch_assembly(cap, nullptr);
                e = hipStreamEndCapture(cap, &g);
                if (e == hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(cap);
            if (e != hipSuccess) {
                P->graph_exec = nullptr;
                return fail(SC_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            }
        }
        HIP_TRY(hipGraphLaunch(P->graph_exec, (hipStream_t)stream));
        P->assembled = true;
        return SC_OK;
    }
    hipEvent_t ev[4];
    hipEvent_t* evp = nullptr;
    if (P->timing) {
        HIP_TRY(P->take_events(4, ev));
        evp = ev;
    }
    HIP_TRY(P->launch_assembly((hipStream_t)stream, evp));
    if (evp && (P->overlapped() || P->arena_elems > 0)) {
        P->pending.push_back({4, ev[0], ev[1]});
        P->event_pool.push_back(ev[2]);
        P->event_pool.push_back(ev[3]);
    } else if (evp) {
        P->pending.push_back({0, ev[0], ev[1]});
        P->pending.push_back({1, ev[2], ev[3]});
    }
    P->assembled = true;
    return SC_OK;
}

static sc_status_t build_implicit(sc_plan_s* P, hipStream_t st);

sc_status_t sc_apply(sc_plan_t P, const double* p_dev, double* q_dev, void* stream) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (!P->assembled) return fail(SC_ERR_STATE, "sc_apply before sc_assemble");
    if (P->dual_total > 0 && (!p_dev || !q_dev)) return fail(SC_ERR_INVALID_ARG, "p or q is NULL");
    if (P->dual_total > 0 && p_dev == q_dev) return fail(SC_ERR_INVALID_ARG, "p and q must not alias");
    HIP_TRY(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    if (P->n_implicit > 0 && !P->impl_ready) {
        const sc_status_t s = build_implicit(P, st);
        if (s != SC_OK) return s;
    }
    hipEvent_t ev[2];
    hipEvent_t* evp = nullptr;
    if (P->timing) {
        HIP_TRY(P->take_events(2, ev));
        evp = ev;
    }
    const DevTables t = P->tables();
    if (evp) HIP_TRY(hipEventRecord(ev[0], st));
    HIP_TRY(launch_apply(t, p_dev, q_dev, st, nullptr));
    // subdomains chosen for the implicit approach (select_iters)
    if (P->n_implicit > 0)
        HIP_TRY(launch_apply_implicit(t, P->ilv_h, P->d_xoff.p, P->d_xwork.p, p_dev, q_dev, P->n_implicit, st, nullptr));
    if (evp) {
        HIP_TRY(hipEventRecord(ev[1], st));
        P->pending.push_back({2, ev[0], ev[1]});
    }
    return SC_OK;
}

sc_status_t sc_apply_noalloc(sc_plan_t P, const double* p_dev, double* q_dev, void* stream) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (!P->assembled) return fail(SC_ERR_STATE, "sc_apply_noalloc before sc_assemble");
    if (P->dual_total > 0 && (!p_dev || !q_dev)) return fail(SC_ERR_INVALID_ARG, "p or q is NULL");
    if (P->dual_total > 0 && p_dev == q_dev) return fail(SC_ERR_INVALID_ARG, "p and q must not alias");
    if (P->n_implicit > 0)
        return fail(SC_ERR_UNSUPPORTED, "sc_apply_noalloc: the plan applies some subdomains implicitly "
                                        "(select_iters); use sc_apply");
    if (P->noalloc_too_big >= 0)
        return fail(SC_ERR_UNSUPPORTED,
                    "sc_apply_noalloc: subdomain " + std::to_string(P->noalloc_too_big) + " has m = " +
                        std::to_string(P->h_subs[P->noalloc_too_big].m) + "; the fixed scratch holds the partial " +
                        "sums of " + std::to_string(kApplyScratchTiles) + " stored F tiles (m <= " +
                        std::to_string(kApplyMaxM) + ")");
    if (P->scratch_err != hipSuccess || !P->scratch)
        return fail(SC_ERR_DEVICE, std::string("sc_apply_noalloc: scratch address: ") +
                                       hipGetErrorString(P->scratch_err));
    HIP_TRY(hipSetDevice(P->device));
    HIP_TRY(launch_apply_chunked(P->tables(), P->h_chunks.data(), (int64_t)P->h_chunks.size(), P->scratch, p_dev,
                                 q_dev, (hipStream_t)stream));
    return SC_OK;
}

sc_status_t sc_pcpg(sc_plan_t P, const double* const* R_host, const int32_t* k_host, const double* d_dev,
                    double* lambda_dev, int32_t iters, double* wnorm_hist, void* stream) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (!P->assembled) return fail(SC_ERR_STATE, "sc_pcpg before sc_assemble");
    if (iters < 0) return fail(SC_ERR_INVALID_ARG, "iters must be >= 0");
    if (P->nsub > 0 && (!R_host || !k_host)) return fail(SC_ERR_INVALID_ARG, "R or k is NULL");
    if (P->dual_total > 0 && (!d_dev || !lambda_dev)) return fail(SC_ERR_INVALID_ARG, "d or lambda is NULL");
    // G_i = B_i R_i and (G_i^T G_i)^{-1} on the host (k_i <= 8)
    std::vector<int64_t> g_off(P->nsub + 1, 0);
    for (int32_t i = 0; i < P->nsub; ++i) {
        if (k_host[i] < 0 || k_host[i] > 8) return fail(SC_ERR_INVALID_ARG, "k_i must be in [0, 8]");
        if (k_host[i] > 0 && !R_host[i]) return fail(SC_ERR_INVALID_ARG, "R_i is NULL");
        g_off[i + 1] = g_off[i] + (int64_t)P->plans[i].m * k_host[i];
    }
    std::vector<double> G((size_t)std::max<int64_t>(1, g_off[P->nsub]));
    std::vector<double> Ginv((size_t)std::max(1, P->nsub) * 64, 0.0);
    for (int32_t i = 0; i < P->nsub; ++i) {
        const SubPlan& sp = P->plans[i];
        const int k = k_host[i];
        const int64_t m = sp.m, n = sp.n;
        double* Gi = G.data() + g_off[i];
        for (int c = 0; c < k; ++c)
            for (int64_t j = 0; j < m; ++j) Gi[c * m + j] = sp.sign[j] * R_host[i][c * n + sp.dof[j]];
        // Gram matrix and its inverse by Gauss-Jordan with partial pivoting
        double A[8][16];
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                double t = 0.0;
                for (int64_t j = 0; j < m; ++j) t += Gi[a * m + j] * Gi[b * m + j];
                A[a][b] = t;
                A[a][k + b] = (a == b) ? 1.0 : 0.0;
            }
        double scale = 0.0;
        for (int a = 0; a < k; ++a) scale = std::max(scale, std::abs(A[a][a]));
        for (int c = 0; c < k; ++c) {
            int piv = c;
            for (int a = c + 1; a < k; ++a)
                if (std::abs(A[a][c]) > std::abs(A[piv][c])) piv = a;
            if (!(std::abs(A[piv][c]) > 1e-13 * scale))
                return fail(SC_ERR_INVALID_ARG, "G^T G of subdomain " + std::to_string(i) + " is singular");
            if (piv != c)
                for (int b = 0; b < 2 * k; ++b) std::swap(A[c][b], A[piv][b]);
            const double inv = 1.0 / A[c][c];
            for (int b = 0; b < 2 * k; ++b) A[c][b] *= inv;
            for (int a = 0; a < k; ++a)
                if (a != c) {
                    const double f = A[a][c];
                    for (int b = 0; b < 2 * k; ++b) A[a][b] -= f * A[c][b];
                }
        }
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) Ginv[(size_t)64 * i + a * k + b] = A[a][k + b];
    }
    HIP_TRY(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    if (P->n_implicit > 0 && !P->impl_ready) {
        const sc_status_t s = build_implicit(P, st);
        if (s != SC_OK) return s;
    }
    // workspace
    const size_t nd = (size_t)std::max<int64_t>(1, P->dual_total);
    DevBuf<double> dG, dGi, dwork, dww, dhist;
    DevBuf<int64_t> doff;
    DevBuf<int32_t> dk;
    auto cleanup = [&]() { dG.release(); dGi.release(); dwork.release(); dww.release(); dhist.release();
                           doff.release(); dk.release(); };
    hipError_t e = dG.alloc(G.size());
    if (e == hipSuccess) e = dGi.alloc(Ginv.size());
    if (e == hipSuccess) e = dwork.alloc(4 * nd);
    if (e == hipSuccess) e = dww.alloc((size_t)std::max(1, P->nsub));
    if (e == hipSuccess && wnorm_hist) e = dhist.alloc((size_t)(iters + 1) * std::max(1, P->nsub));
    if (e == hipSuccess) e = doff.alloc(g_off.size());
    if (e == hipSuccess) e = dk.alloc((size_t)std::max(1, P->nsub));
    if (e == hipSuccess) e = hipMemcpyAsync(dG.p, G.data(), G.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dGi.p, Ginv.data(), Ginv.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(doff.p, g_off.data(), g_off.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && P->nsub > 0) e = hipMemcpyAsync(dk.p, k_host, (size_t)P->nsub * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        PcpgArgs a;
        a.G = dG.p; a.g_off = doff.p; a.kdim = dk.p; a.GtGinv = dGi.p;
        a.d = d_dev; a.lambda = lambda_dev;
        a.r = dwork.p; a.w = dwork.p + nd; a.p = dwork.p + 2 * nd; a.q = dwork.p + 3 * nd;
        a.ww = dww.p; a.hist = dhist.p; a.nsub = P->nsub; a.iters = iters;
        e = launch_pcpg(P->tables(), a, st, P->n_implicit > 0 ? &P->ilv_h : nullptr, P->d_xoff.p, P->d_xwork.p,
                        P->n_implicit);
    }
    if (e == hipSuccess && wnorm_hist)
        e = hipMemcpyAsync(wnorm_hist, dhist.p, (size_t)(iters + 1) * P->nsub * 8, hipMemcpyDeviceToHost, st);
    // the workspace is released after the queued work has finished
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? SC_ERR_OOM : SC_ERR_DEVICE,
                                     std::string("sc_pcpg: ") + hipGetErrorString(e));
    return SC_OK;
}

// Level schedule and workspace of the implicit apply, built on first use:
// everything goes into locals and is committed to the plan only when every
// allocation, copy and the final synchronisation succeeded (a failed attempt
// leaves the plan as it was and releases what it allocated).
static sc_status_t build_implicit(sc_plan_s* P, hipStream_t st) {
    std::vector<int64_t> off(P->nsub + 1, 0);
    for (int32_t i = 0; i < P->nsub; ++i) off[i + 1] = off[i] + P->plans[i].n;
    // levels: forward = 1 + max over the blocks whose pruned rows reach the
    // block; backward = 1 + max over the blocks the block's pruned rows lie in
    std::vector<std::vector<int2>> fw, bw;
    std::vector<int64_t> rptr_off(P->nsub, 0);
    std::vector<int32_t> rptr, rpos;
    int64_t nblocks_all = 0, nlevels_all = 0, nlevels_sub_h = 0;
    std::vector<int64_t> sub_levels(P->nsub, 0);
    for (int32_t i = 0; i < P->nsub; ++i) {
        const SubPlan& sp = P->plans[i];
        const SubDev& sd = P->h_subs[i];
        const int32_t nb = (int32_t)sp.blocks.size();
        std::vector<int32_t> lf(nb, 0), lb(nb, 0);
        for (int32_t b = 0; b < nb; ++b) {
            const BlockDesc& d = sp.blocks[b];
            for (int32_t q = 0; q < d.nbelow; ++q) {
                const int32_t t = sp.block_of_row[sp.brows[d.rows_off + q]];
                lf[t] = std::max(lf[t], lf[b] + 1);
            }
        }
        for (int32_t b = nb - 1; b >= 0; --b) {
            const BlockDesc& d = sp.blocks[b];
            for (int32_t q = 0; q < d.nbelow; ++q)
                lb[b] = std::max(lb[b], lb[sp.block_of_row[sp.brows[d.rows_off + q]]] + 1);
        }
        nblocks_all += nb;
        sub_levels[i] = nb > 0 ? 1 + *std::max_element(lf.begin(), lf.end()) : 0;
        nlevels_all += sub_levels[i];
        for (int32_t b = 0; b < nb; ++b) {
            if ((size_t)lf[b] >= fw.size()) fw.resize(lf[b] + 1);
            if ((size_t)lb[b] >= bw.size()) bw.resize(lb[b] + 1);
            fw[lf[b]].push_back(make_int2(i, b));
            bw[lb[b]].push_back(make_int2(i, b));
        }
        // per row: positions (in the global row array) where it is a pruned row
        std::vector<int32_t> cnt(sp.n + 1, 0);
        for (int32_t b = 0; b < nb; ++b) {
            const BlockDesc& d = sp.blocks[b];
            for (int32_t q = 0; q < d.nbelow; ++q) ++cnt[sp.brows[d.rows_off + q] + 1];
        }
        for (int32_t r = 0; r < sp.n; ++r) cnt[r + 1] += cnt[r];
        rptr_off[i] = (int64_t)rptr.size();
        const int32_t base = (int32_t)rpos.size();
        for (int32_t r = 0; r <= sp.n; ++r) rptr.push_back(base + cnt[r]);
        rpos.resize(rpos.size() + cnt[sp.n]);
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for (int32_t b = 0; b < nb; ++b) {             // increasing source block: fixed order
            const BlockDesc& d = sp.blocks[b];
            for (int32_t q = 0; q < d.nbelow; ++q)
                rpos[base + fill[sp.brows[d.rows_off + q]]++] = (int32_t)(sd.rows_off + d.rows_off + q);
        }
    }
    std::vector<int2> fwi, bwi;
    ImplicitLevels lv;
    lv.fw_off.assign(1, 0);
    lv.bw_off.assign(1, 0);
    for (auto& l : fw) { fwi.insert(fwi.end(), l.begin(), l.end()); lv.fw_off.push_back((int64_t)fwi.size()); }
    for (auto& l : bw) { bwi.insert(bwi.end(), l.begin(), l.end()); lv.bw_off.push_back((int64_t)bwi.size()); }
    // the subset applied implicitly next to the assembled subdomains
    std::vector<int2> fwh, bwh;
    std::vector<int32_t> impl_list;
    ImplicitLevels lvh;
    lvh.fw_off.assign(1, 0);
    lvh.bw_off.assign(1, 0);
    int64_t nblocks_h = 0;
    for (int32_t i = 0; i < P->nsub; ++i)
        if (P->implicit_sub[i]) {
            impl_list.push_back(i);
            nblocks_h += (int64_t)P->plans[i].blocks.size();
            nlevels_sub_h += sub_levels[i];
        }
    auto subset = [&](const std::vector<std::vector<int2>>& lev, std::vector<int2>& out, std::vector<int64_t>& off) {
        for (auto& l : lev) {
            for (const int2& it : l)
                if (P->implicit_sub[it.x]) out.push_back(it);
            if ((int64_t)out.size() > off.back()) off.push_back((int64_t)out.size());
        }
    };
    subset(fw, fwh, lvh.fw_off);
    subset(bw, bwh, lvh.bw_off);
    DevBuf<double> xwork, ywork, ubuf;
    DevBuf<int64_t> xoff, rptr_off_d;
    DevBuf<int2> ifw, ibw;
    DevBuf<int32_t> rptr_d, rpos_d;
    DevBuf<int2> ifwh, ibwh;
    DevBuf<int32_t> ilist;
    auto release_all = [&]() {
        xwork.release(); ywork.release(); ubuf.release(); xoff.release(); rptr_off_d.release();
        ifw.release(); ibw.release(); rptr_d.release(); rpos_d.release();
        ifwh.release(); ibwh.release(); ilist.release();
    };
    hipError_t e = xwork.alloc((size_t)off[P->nsub]);
    if (e == hipSuccess) e = ywork.alloc((size_t)off[P->nsub]);
    if (e == hipSuccess) e = xoff.alloc(off.size());
    if (e == hipSuccess) e = ifw.alloc(std::max<size_t>(1, fwi.size()));
    if (e == hipSuccess) e = ibw.alloc(std::max<size_t>(1, bwi.size()));
    if (e == hipSuccess) e = rptr_off_d.alloc(rptr_off.size());
    if (e == hipSuccess) e = rptr_d.alloc(rptr.size());
    if (e == hipSuccess) e = rpos_d.alloc(std::max<size_t>(1, rpos.size()));
    if (e == hipSuccess) e = ubuf.alloc((size_t)P->nrows_total);
    if (e == hipSuccess) e = ifwh.alloc(fwh.size());
    if (e == hipSuccess) e = ibwh.alloc(bwh.size());
    if (e == hipSuccess) e = ilist.alloc(impl_list.size());
    auto up = [&](void* d, const void* h, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    if (e == hipSuccess) e = up(xoff.p, off.data(), off.size() * 8);
    if (e == hipSuccess) e = up(ifw.p, fwi.data(), fwi.size() * sizeof(int2));
    if (e == hipSuccess) e = up(ibw.p, bwi.data(), bwi.size() * sizeof(int2));
    if (e == hipSuccess) e = up(rptr_off_d.p, rptr_off.data(), rptr_off.size() * 8);
    if (e == hipSuccess) e = up(rptr_d.p, rptr.data(), rptr.size() * 4);
    if (e == hipSuccess) e = up(rpos_d.p, rpos.data(), rpos.size() * 4);
    if (e == hipSuccess) e = up(ifwh.p, fwh.data(), fwh.size() * sizeof(int2));
    if (e == hipSuccess) e = up(ibwh.p, bwh.data(), bwh.size() * sizeof(int2));
    if (e == hipSuccess) e = up(ilist.p, impl_list.data(), impl_list.size() * 4);
    if (e == hipSuccess) e = hipStreamSynchronize(st);    // the host tables go out of scope
    if (e != hipSuccess) {
        release_all();
        return fail(e == hipErrorOutOfMemory ? SC_ERR_OOM : SC_ERR_DEVICE,
                    std::string("implicit apply setup: ") + hipGetErrorString(e));
    }
    lv.fw_items = ifw.p;
    lv.bw_items = ibw.p;
    lv.rptr_off = rptr_off_d.p;
    lv.rptr = rptr_d.p;
    lv.rpos = rpos_d.p;
    lv.ubuf = ubuf.p;
    lv.ywork = ywork.p;
    // near-chain block DAGs (fewer than 1.5 blocks per level): a level
    // launch would carry one block per subdomain
    lv.per_subdomain = 2 * nblocks_all < 3 * nlevels_all;
    P->d_xwork = xwork; P->d_ywork = ywork; P->d_xoff = xoff; P->d_ifw = ifw; P->d_ibw = ibw;
    P->d_rptr_off = rptr_off_d; P->d_rptr = rptr_d; P->d_rpos = rpos_d; P->d_ubuf = ubuf;
    P->ilv = lv;
    lvh.fw_items = ifwh.p;
    lvh.bw_items = ibwh.p;
    lvh.rptr_off = lv.rptr_off;
    lvh.rptr = lv.rptr;
    lvh.rpos = lv.rpos;
    lvh.ubuf = lv.ubuf;
    lvh.ywork = lv.ywork;
    lvh.subs = ilist.p;
    // per-subdomain sweeps for the subset when its own block DAGs are near
    // chains (the per-subdomain kernel reads the list)
    lvh.per_subdomain = 2 * nblocks_h < 3 * nlevels_sub_h;
    P->d_ifw_h = ifwh; P->d_ibw_h = ibwh; P->d_impl_list = ilist;
    P->ilv_h = lvh;
    P->impl_ready = true;
    return SC_OK;
}

sc_status_t sc_apply_implicit(sc_plan_t P, const double* p_dev, double* q_dev, void* stream) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (!P->factored) return fail(SC_ERR_STATE, "sc_apply_implicit before sc_factor");
    if (P->dual_total > 0 && (!p_dev || !q_dev)) return fail(SC_ERR_INVALID_ARG, "p or q is NULL");
    if (P->dual_total > 0 && p_dev == q_dev) return fail(SC_ERR_INVALID_ARG, "p and q must not alias");
    HIP_TRY(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    if (P->nsub == 0) return SC_OK;
    if (!P->impl_ready) {
        const sc_status_t s = build_implicit(P, st);
        if (s != SC_OK) return s;
    }
    const DevTables t = P->tables();
    if (P->opt.use_graph && !P->timing) {
        // the triangular sweeps read and write only plan-owned buffers: they
        // are captured once and replayed for every call; the scatter of p and
        // the gather into q run eagerly around the replay
        if (!P->impl_graph) {
            hipStream_t cap;
            HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t el = launch_implicit_sweeps(t, P->ilv, P->d_xoff.p, P->d_xwork.p, P->nsub, cap);
                e = hipStreamEndCapture(cap, &g);
                if (e == hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(cap);
            if (e != hipSuccess) return fail(SC_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            P->impl_graph = ex;
        }
        HIP_TRY(launch_implicit_init(t, P->d_xoff.p, P->d_xwork.p, p_dev, nullptr, P->nsub, st));
        HIP_TRY(hipGraphLaunch(P->impl_graph, st));
        HIP_TRY(launch_implicit_gather(t, P->d_xoff.p, P->d_xwork.p, q_dev, nullptr, P->nsub, st));
        return SC_OK;
    }
    hipEvent_t ev[2];
    hipEvent_t* evp = nullptr;
    if (P->timing) {
        HIP_TRY(P->take_events(2, ev));
        evp = ev;
    }
    HIP_TRY(launch_apply_implicit(t, P->ilv, P->d_xoff.p, P->d_xwork.p, p_dev, q_dev, P->nsub, st, evp));
    if (evp) P->pending.push_back({3, ev[0], ev[1]});
    return SC_OK;
}

sc_status_t sc_get_F(sc_plan_t P, int32_t sub, double* out, int32_t ld, int32_t on_device, void* stream) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (sub < 0 || sub >= P->nsub) return fail(SC_ERR_INVALID_ARG, "subdomain index out of range");
    if (!P->assembled) return fail(SC_ERR_STATE, "sc_get_F before sc_assemble");
    if (P->implicit_sub[sub])
        return fail(SC_ERR_STATE, "subdomain " + std::to_string(sub) + " is applied implicitly (select_iters): "
                                  "its F is not assembled");
    const SubDev& s = P->h_subs[sub];
    if (s.m == 0) return SC_OK;
    if (!out || ld < s.m) return fail(SC_ERR_INVALID_ARG, "bad output buffer or ld");
    HIP_TRY(hipSetDevice(P->device));
    hipStream_t st = (hipStream_t)stream;
    // packed lower tiles in sorted column order -> dense, original order
    const int64_t m = s.m;
    const int64_t nt = (m + kSyrkTile - 1) / kSyrkTile;
    const size_t cnt = (size_t)(nt * (nt + 1) / 2) * kFTileElems;
    std::vector<double> tiles(cnt);
    if (!P->mixed) {
        HIP_TRY(hipMemcpyAsync(tiles.data(), P->d_F.p + s.F_off, cnt * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    } else {
        std::vector<float> t32(cnt);
        HIP_TRY(hipMemcpyAsync(t32.data(), P->d_F32.p + s.F_off, cnt * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (size_t k = 0; k < cnt; ++k) tiles[k] = (double)t32[k];
    }
    const std::vector<int32_t>& pi = P->plans[sub].pi;
    std::vector<double> dense((size_t)m * m);
    for (int64_t b = 0; b < m; ++b)
        for (int64_t a = 0; a < m; ++a) {
            int64_t hi = a, lo = b;                 // (hi, lo) lies in a stored tile
            if (a / kSyrkTile < b / kSyrkTile) std::swap(hi, lo);
            const int64_t I = hi / kSyrkTile, J = lo / kSyrkTile;
            dense[(size_t)pi[b] * m + pi[a]] =
                tiles[(size_t)(I * (I + 1) / 2 + J) * kFTileElems + (hi % kSyrkTile) * kSyrkTile + lo % kSyrkTile];
        }
    if (on_device) {
        HIP_TRY(hipMemcpy2DAsync(out, (size_t)ld * sizeof(double), dense.data(), (size_t)m * sizeof(double),
                                 (size_t)m * sizeof(double), (size_t)m, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    } else {
        for (int64_t c = 0; c < m; ++c) std::copy(dense.begin() + c * m, dense.begin() + (c + 1) * m, out + c * ld);
    }
    return SC_OK;
}

sc_status_t sc_query(sc_plan_t P, int32_t sub, int64_t* n, int64_t* m, int64_t* dual_offset, int64_t* nnzL,
                     double* useful_flops) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (sub < 0 || sub >= P->nsub) return fail(SC_ERR_INVALID_ARG, "subdomain index out of range");
    const SubPlan& sp = P->plans[sub];
    if (n) *n = sp.n;
    if (m) *m = sp.m;
    if (dual_offset) *dual_offset = P->h_subs[sub].dual_off;
    if (nnzL) *nnzL = sp.nnzL;
    if (useful_flops) *useful_flops = sp.trsm_useful + sp.syrk_useful;
    return SC_OK;
}

sc_status_t sc_query_selection(sc_plan_t P, int32_t sub, int32_t* implicit, double* t_asm_ms, double* t_expl_ms,
                               double* t_impl_ms, double* n_star) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (sub < 0 || sub >= P->nsub) return fail(SC_ERR_INVALID_ARG, "subdomain index out of range");
    const Prediction& q = P->pred[sub];
    if (implicit) *implicit = P->implicit_sub[sub];
    if (t_asm_ms) *t_asm_ms = q.t_asm_ms;
    if (t_expl_ms) *t_expl_ms = q.t_expl_ms;
    if (t_impl_ms) *t_impl_ms = q.t_impl_ms;
    if (n_star) *n_star = q.n_star;
    return SC_OK;
}

sc_status_t sc_plan_stats(sc_plan_t P, int32_t* nsub, int64_t* dual_total, double* trsm_useful,
                          double* syrk_useful, double* trsm_dense, double* syrk_dense,
                          double* trsm_reach, double* syrk_reach, int64_t* device_bytes) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    if (nsub) *nsub = P->nsub;
    if (dual_total) *dual_total = P->dual_total;
    if (trsm_useful) *trsm_useful = P->trsm_u;
    if (syrk_useful) *syrk_useful = P->syrk_u;
    if (trsm_dense) *trsm_dense = P->trsm_d;
    if (syrk_dense) *syrk_dense = P->syrk_d;
    if (trsm_reach) *trsm_reach = P->trsm_r;
    if (syrk_reach) *syrk_reach = P->syrk_r;
    if (device_bytes) *device_bytes = P->device_bytes();
    return SC_OK;
}

sc_status_t sc_host_analyze(const sc_subdomain_desc_t* sd, const sc_options_t* opt, const double* kreg_vals,
                            int32_t* perm_out, double* L_out, int32_t* piv_out, int32_t* pi_out,
                            sc_host_info_t* info, int32_t* failed_col) {
    g_last_error.clear();
    if (!sd) return fail(SC_ERR_INVALID_ARG, "descriptor is NULL");
    sc_options_t o{};
    if (opt) o = *opt;
    PlanOptions po;
    std::string err = to_plan_options(o, po);
    if (!err.empty()) return fail(SC_ERR_INVALID_ARG, err);
    if (L_out && (!kreg_vals || sd->n > 4096)) return fail(SC_ERR_INVALID_ARG, "dense L needs values and n <= 4096");
    SubPlan sp;
    int code = 0;
    try {
        err = plan_subdomain(*sd, po, o.lower_only_csr != 0, sp, code);
    } catch (const std::bad_alloc&) {
        return fail(SC_ERR_OOM, "host allocation failed");
    }
    if (!err.empty()) return fail(SC_ERR_INVALID_ARG, err);
    if (perm_out) std::copy(sp.perm.begin(), sp.perm.end(), perm_out);
    if (piv_out) std::copy(sp.piv.begin(), sp.piv.end(), piv_out);
    if (pi_out) std::copy(sp.pi.begin(), sp.pi.end(), pi_out);
    if (info) {
        sc_host_info_t h{};
        h.n = sp.n;
        h.m = sp.m;
        h.nnzL = sp.nnzL;
        h.nnzL_stored = sp.nnzL_stored;
        h.nsuper = sp.nsuper;
        h.nblocks = (int64_t)sp.blocks.size();
        for (int32_t s = 0; s < sp.nsuper; ++s)
            h.max_width = std::max<int64_t>(h.max_width, sp.sfirst[s + 1] - sp.sfirst[s]);
        for (const BlockDesc& b : sp.blocks) h.sum_below += b.nbelow;
        h.trsm_useful = sp.trsm_useful;
        h.syrk_useful = sp.syrk_useful;
        h.trsm_dense = sp.trsm_dense;
        h.syrk_dense = sp.syrk_dense;
        h.factor_flops = sp.factor_flops;
        h.trsm_reach = sp.trsm_reach;
        h.syrk_reach = sp.syrk_reach;
        h.trsm_visits = (int64_t)sp.visit.size();
        h.stair_visits = sp.visits_stair;
        const Prediction q = predict(sp, o.precision == SC_PREC_MIXED, o);
        h.t_asm_ms = q.t_asm_ms;
        h.t_expl_ms = q.t_expl_ms;
        h.t_impl_ms = q.t_impl_ms;
        h.n_star = q.n_star;
        for (int64_t k = 0; k < (int64_t)sp.visit.size(); ++k) h.pruned_updates += sp.blocks[sp.visit[k]].nbelow;
        if (!o.disable_pair_merge) {
            const std::vector<int32_t> pair = merge_pairs(sp);
            for (int32_t f : pair) h.merge_pairs += f;
            const int32_t ntile = (sp.m + kTile - 1) / kTile;
            for (int32_t t = 0; t < ntile; ++t)
                for (int64_t k = sp.visit_ptr[t]; k + 1 < sp.visit_ptr[t + 1]; ++k) {
                    const int32_t b = sp.visit[k];
                    if (pair[b] && sp.visit[k + 1] == b + 1) h.merged_rows += sp.blocks[b + 1].nbelow;
                }
        }
        *info = h;
    }
    if (kreg_vals) {
        std::vector<double> vals((size_t)std::max<int64_t>(1, sp.nval));
        const int64_t bad = factor_numeric(sp, kreg_vals, vals.data());
        if (bad >= 0) {
            if (failed_col) *failed_col = (int32_t)bad;
            return fail(SC_ERR_NOT_SPD, "pivot of permuted column " + std::to_string(bad) + " is not positive");
        }
        if (L_out) {
            const int64_t n = sp.n;
            std::fill(L_out, L_out + n * n, 0.0);
            for (int32_t s = 0; s < sp.nsuper; ++s) {
                const int32_t f = sp.sfirst[s], w = sp.sfirst[s + 1] - f;
                const int64_t ld = sp.srow_ptr[s + 1] - sp.srow_ptr[s];
                const int32_t* rows = sp.srows.data() + sp.srow_ptr[s];
                const double* A = vals.data() + sp.spanel_off[s];
                for (int32_t c = 0; c < w; ++c)
                    for (int64_t q = c; q < ld; ++q) L_out[(int64_t)rows[q] * n + f + c] = A[c * ld + q];
            }
        }
    }
    return SC_OK;
}

sc_status_t sc_host_tile_visits(const sc_subdomain_desc_t* sd, const sc_options_t* opt, int64_t* counts,
                                int32_t* block_row0, int64_t* visit_ptr, int32_t* visit, int64_t capacity,
                                uint64_t* step_mask) {
    g_last_error.clear();
    if (!sd || !counts) return fail(SC_ERR_INVALID_ARG, "descriptor or counts is NULL");
    sc_options_t o{};
    if (opt) o = *opt;
    PlanOptions po;
    std::string err = to_plan_options(o, po);
    if (!err.empty()) return fail(SC_ERR_INVALID_ARG, err);
    SubPlan sp;
    int code = 0;
    try {
        err = plan_subdomain(*sd, po, o.lower_only_csr != 0, sp, code);
    } catch (const std::bad_alloc&) {
        return fail(SC_ERR_OOM, "host allocation failed");
    }
    if (!err.empty()) return fail(SC_ERR_INVALID_ARG, err);
    const int64_t nb = (int64_t)sp.blocks.size(), total = (int64_t)sp.visit.size();
    counts[0] = nb;
    counts[1] = (int64_t)sp.visit_ptr.size() - 1;
    counts[2] = total;
    counts[3] = sp.mask_words;
    if (step_mask) std::copy(sp.step_mask.begin(), sp.step_mask.end(), step_mask);
    if (block_row0) {
        for (int64_t b = 0; b < nb; ++b) block_row0[b] = sp.blocks[b].row0;
        block_row0[nb] = sp.n;
    }
    if (visit_ptr) std::copy(sp.visit_ptr.begin(), sp.visit_ptr.end(), visit_ptr);
    if (visit) {
        if (capacity < total) return fail(SC_ERR_INVALID_ARG, "visit capacity below the total visit count");
        std::copy(sp.visit.begin(), sp.visit.end(), visit);
    }
    return SC_OK;
}

sc_status_t sc_set_timing(sc_plan_t P, int32_t enable) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    P->timing = enable != 0;
    return SC_OK;
}

sc_status_t sc_kernel_times(sc_plan_t P, double* ms, int64_t* counts, int32_t reset) {
    g_last_error.clear();
    if (!P) return fail(SC_ERR_INVALID_ARG, "plan is NULL");
    HIP_TRY(hipSetDevice(P->device));
    HIP_TRY(P->drain_timing(true));
    for (int k = 0; k < kNumTimed; ++k) {
        if (ms) ms[k] = P->ms_sum[k];
        if (counts) counts[k] = P->ms_count[k];
        if (reset) { P->ms_sum[k] = 0; P->ms_count[k] = 0; }
    }
    return SC_OK;
}

sc_status_t sc_autotune(const sc_subdomain_desc_t* sd, int32_t nsub, const sc_options_t* base,
                        const double* const* kreg_vals, const int32_t* candidates, int32_t ncand,
                        int32_t sample, int32_t reps, void* stream, int32_t* best_width, double* times_ms) {
    g_last_error.clear();
    if (!sd || nsub <= 0 || !kreg_vals || !candidates || ncand <= 0 || !best_width || reps < 1)
        return fail(SC_ERR_INVALID_ARG, "bad autotune arguments");
    for (int32_t c = 0; c < ncand; ++c)
        if (candidates[c] < 16 || candidates[c] > kMaxPanel)
            return fail(SC_ERR_INVALID_ARG, "candidate width out of [16, 64]");
    // size-stratified sample
    std::vector<int32_t> idx(nsub);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return sd[a].n < sd[b].n; });
    const int32_t ns = std::max(1, std::min(sample > 0 ? sample : nsub, nsub));
    std::vector<sc_subdomain_desc_t> sub(ns);
    std::vector<const double*> vals(ns);
    for (int32_t k = 0; k < ns; ++k) {
        const int32_t i = idx[(int64_t)k * nsub / ns];
        sub[k] = sd[i];
        vals[k] = kreg_vals[i];
    }
    sc_options_t o{};
    if (base) o = *base;
    o.use_graph = 0;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e300;
    sc_status_t status = SC_OK;
    for (int32_t c = 0; c < ncand && status == SC_OK; ++c) {
        o.panel_width = candidates[c];
        sc_plan_t P = nullptr;
        status = sc_plan_create(sub.data(), ns, &o, stream, &P);
        if (status == SC_OK) status = sc_factor(P, vals.data(), stream, nullptr, nullptr);
        if (status == SC_OK) status = sc_assemble(P, stream);          // warm-up
        float ms = 0.f;
        if (status == SC_OK) {
            hipError_t e = hipEventRecord(e0, st);
            for (int32_t r = 0; r < reps && e == hipSuccess; ++r)
                if (sc_assemble(P, stream) != SC_OK) e = hipErrorUnknown;
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) status = fail(SC_ERR_DEVICE, "autotune timing failed");
        }
        const std::string keep = g_last_error;
        sc_plan_destroy(P);
        g_last_error = keep;
        if (status != SC_OK) break;
        const double t = ms / reps;
        if (times_ms) times_ms[c] = t;
        if (t < best) {
            best = t;
            *best_width = candidates[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

sc_status_t sc_autotune_classes(const sc_subdomain_desc_t* sd, int32_t nsub, const sc_options_t* base,
                                const double* const* kreg_vals, int32_t sample, int32_t reps,
                                const char* cache_path, void* stream, sc_tune_class_t* classes,
                                int32_t max_classes, int32_t* nclasses) {
    g_last_error.clear();
    if (!sd || nsub <= 0 || !kreg_vals || sample < 1 || reps < 1 || !classes || max_classes < 1 || !nclasses)
        return fail(SC_ERR_INVALID_ARG, "bad autotune arguments");
    sc_options_t o0{};
    if (base) o0 = *base;
    o0.use_graph = 0;
    o0.tune_classes = nullptr;
    o0.ntune_classes = 0;
    const char* prec = o0.precision == SC_PREC_MIXED ? "mixed" : "fp64";
    // size classes [0, 1024), [1024, 2048), [2048, 4096), ...; the last one open
    auto class_of = [](int32_t n) {
        int c = 0;
        while (c < 20 && n >= (1 << (c + 10))) ++c;
        return c;
    };
    std::vector<std::vector<int32_t>> members(21);
    for (int32_t i = 0; i < nsub; ++i) members[class_of(sd[i].n)].push_back(i);
    std::vector<int> used;
    for (int c = 0; c <= 20; ++c)
        if (!members[c].empty()) used.push_back(c);
    if ((int32_t)used.size() > max_classes)
        return fail(SC_ERR_INVALID_ARG, "max_classes = " + std::to_string(max_classes) + " < " +
                                            std::to_string(used.size()) + " size classes");
    const std::string dev = device_key();
    // cached classes
    struct Cached { int32_t lo, hi, pw, split, syrk; float ms; };
    std::vector<Cached> cached;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "r");
        if (f) {
            char line[512];
            while (std::fgets(line, sizeof line, f)) {
                if (line[0] == '#') continue;
                char d[256], pr[16];
                Cached k{};
                if (std::sscanf(line, "%255s %15s %d %d %d %d %d %f", d, pr, &k.lo, &k.hi, &k.pw, &k.split, &k.syrk,
                                &k.ms) == 8 &&
                    dev == d && std::strcmp(pr, prec) == 0)
                    cached.push_back(k);
            }
            std::fclose(f);
        }
    }
    hipStream_t st = (hipStream_t)stream;
    (void)st;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    sc_status_t status = SC_OK;
    std::vector<std::string> fresh;
    int32_t nc = 0;
    for (size_t u = 0; u < used.size() && status == SC_OK; ++u) {
        const int c = used[u];
        const int32_t lo = c == 0 ? 0 : (1 << (c + 9));
        const int32_t hi = u + 1 == used.size() ? INT32_MAX : (1 << (c + 10));
        sc_tune_class_t out{lo, hi, 64, 0, 0, 0.f};
        bool hit = false;
        for (const Cached& k : cached)
            if (k.lo == lo && k.hi == hi) {
                out = sc_tune_class_t{lo, hi, k.pw, k.split, k.syrk, k.ms};
                hit = true;
                break;
            }
        if (!hit) {
            std::vector<int32_t> idx = members[c];
            std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return sd[a].n < sd[b].n; });
            const int32_t ns = std::min<int32_t>(sample, (int32_t)idx.size());
            std::vector<sc_subdomain_desc_t> sub(ns);
            std::vector<const double*> vals(ns);
            for (int32_t k = 0; k < ns; ++k) {
                const int32_t i = idx[(int64_t)k * (int64_t)idx.size() / ns];
                sub[k] = sd[i];
                vals[k] = kreg_vals[i];
            }
            auto run = [&](int32_t pw, int32_t split, int32_t syrk, double* ms) {
                sc_options_t o = o0;
                sc_tune_class_t one{0, INT32_MAX, pw, split, syrk, 0.f};
                o.tune_classes = &one;
                o.ntune_classes = 1;
                return time_candidate(sub.data(), ns, o, vals.data(), reps, stream, e0, e1, ms);
            };
            // SYRK kind the size rule gives this class's largest sample member
            const int32_t nmax = sub[ns - 1].n;
            const int32_t by_size = nmax <= (o0.precision == SC_PREC_MIXED ? kSyrkBlockMaxNMixed : kSyrkBlockMaxN) ? 1 : 2;
            double best = 0.0, t = 0.0;
            status = run(64, 0, by_size, &best);
            out.panel_width = 64;
            out.block_split = 0;
            out.syrk_kind = by_size;
            if (status == SC_OK && (status = run(64, 1, by_size, &t)) == SC_OK && t < best) {
                best = t;
                out.block_split = 1;
            }
            for (int32_t pw : {32, 48}) {
                if (status != SC_OK) break;
                if ((status = run(pw, out.block_split, by_size, &t)) == SC_OK && t < best) {
                    best = t;
                    out.panel_width = pw;
                }
            }
            if (status == SC_OK && (status = run(out.panel_width, out.block_split, 3 - by_size, &t)) == SC_OK &&
                t < best) {
                best = t;
                out.syrk_kind = 3 - by_size;
            }
            out.ms_per_sub = (float)(best / ns);
            char line[512];
            std::snprintf(line, sizeof line, "%s %s %d %d %d %d %d %.6g\n", dev.c_str(), prec, lo, hi,
                          out.panel_width, out.block_split, out.syrk_kind, (double)out.ms_per_sub);
            fresh.push_back(line);
        }
        classes[nc++] = out;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != SC_OK) return status;
    *nclasses = nc;
    if (cache_path && !fresh.empty()) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(SC_ERR_DEVICE, std::string("cannot write the autotune cache ") + cache_path);
        for (const std::string& l : fresh) std::fputs(l.c_str(), f);
        std::fclose(f);
    }
    return SC_OK;
}

sc_status_t sc_plan_destroy(sc_plan_t P) {
    if (!P) return SC_OK;
    (void)hipSetDevice(P->device);
    // queued work may still use the plan's buffers and graphs
    (void)hipDeviceSynchronize();
    P->release();
    delete P;
    return SC_OK;
}

}  // extern "C"
