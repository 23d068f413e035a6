/*
 * scasm -- sparsity-aware assembly of FETI dual Schur complements on AMD
 * MI355X (gfx950).  C ABI of libscasm.so.
 *
 * The library assembles, for a batch of subdomains i, the dense local dual
 * operator (paper, Sec. 2.1 eq. (9) and Sec. 2.2 eq. (10))
 *
 *     F_i = B_i K_i^+ B_i^T = B_i K_reg,i^{-1} B_i^T = Y_i^T Y_i,
 *     Y_i = L_i^{-1} P_i B_i^T,   L_i L_i^T = P_i K_reg,i P_i^T,
 *
 * (the SYRK form of Sec. 3.1, eq. (14)), from a CPU-computed sparse Cholesky
 * factor L_i and the signed-boolean gluing matrix B_i, and applies it
 * (Sec. 2.2, eqs. (11)-(12)).  The three solver stages of Sec. 2.2 map to
 *     initialisation  -> sc_plan_create   (ordering, symbolic factorisation,
 *                                          staircase plan, device buffers)
 *     preprocessing   -> sc_factor + sc_assemble, or sc_preprocess (both,
 *                        pipelined: host factorisation overlapped with the
 *                        GPU assembly, Sec. 4.4)
 *     solution        -> sc_apply (explicit, eq. (12)) or
 *                        sc_apply_implicit (eq. (11))
 *
 * Conventions
 *   - Host arrays passed in are borrowed for the duration of the call only.
 *   - Device pointers (p_dev, q_dev, ...) are caller-owned HIP device memory.
 *   - `stream` is a hipStream_t passed as void*; NULL = the null stream.
 *   - Every function returns an sc_status_t; no C++ exception crosses the ABI.
 *     sc_last_error() returns a thread-local message for the last failure.
 *   - Asynchronous calls report launch errors at once; execution errors
 *     surface at the next synchronising call.
 *   - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef SCASM_H
#define SCASM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_plan_s* sc_plan_t;

typedef enum {
    SC_OK = 0,
    SC_ERR_INVALID_ARG = 1,   /* bad size, index, sign, pointer or option      */
    SC_ERR_NOT_SPD = 2,       /* a Cholesky pivot of K_reg was not positive    */
    SC_ERR_OOM = 3,           /* device or host allocation failed              */
    SC_ERR_DEVICE = 4,        /* a HIP call failed (message in sc_last_error)  */
    SC_ERR_UNSUPPORTED = 5,   /* option combination not implemented            */
    SC_ERR_STATE = 6          /* call out of order (e.g. assemble before factor) */
} sc_status_t;

typedef enum {
    SC_PREC_FP64 = 0,         /* every step in FP64; F stored FP64 */
    SC_PREC_MIXED = 1         /* FP64 diagonal-block solves; FP32 off-diagonal
                                 updates, X and SYRK (FP32 MFMA, FP32 accumulate);
                                 F stored FP32 */
} sc_precision_t;

/*
 * One subdomain (paper, Sec. 3: "the input for the algorithm is B^T together
 * with the factor L", L of the fill-reduced K_reg).
 *   n              DOFs (> 0)
 *   kreg_rowptr    [n+1] int64 CSR row pointers of K_reg (both triangles, or
 *                  the lower one with sc_options_t::lower_only_csr)
 *   kreg_col       column indices; the pattern is fixed for the plan's life
 *   m              multipliers = columns of B^T (>= 0)
 *   bt_dof         [m] DOF (original numbering) of column j's single nonzero
 *   bt_sign        [m] its value, +1 or -1
 *   perm           optional [n] fill-reducing order, perm[new] = old; NULL =
 *                  the library's nested dissection
 *   coords         optional [n/dofs_per_node][dim] node coordinates for the
 *                  geometric nested dissection; NULL = graph (BFS) dissection
 *   dim            coordinate dimension (with coords)
 *   dofs_per_node  1 (heat) or 3 (elasticity); DOFs of a node are contiguous
 */
typedef struct {
    int32_t n;
    const int64_t* kreg_rowptr;
    const int32_t* kreg_col;
    int32_t m;
    const int32_t* bt_dof;
    const int8_t* bt_sign;
    const int32_t* perm;
    const double* coords;
    int32_t dim;
    int32_t dofs_per_node;
} sc_subdomain_desc_t;

/*
 * Options; zero-initialised = defaults.
 *   precision        SC_PREC_FP64 / SC_PREC_MIXED
 *   staircase        1 (default when 0 is not forced) = sort the columns of
 *                    B^T by pivot and skip the zero trapezoid of X (Sec. 3.2,
 *                    3.3); set disable_staircase = 1 for the plain ("orig",
 *                    Sec. 3.1) assembly that skips nothing
 *   panel_width      GPU factor blocks: supernodes split into panels of at
 *                    most this many columns (Sec. 3.2, factor splitting;
 *                    default 64)
 *   relax_width      relaxed supernode amalgamation bound (default 64)
 *   leaf_nodes       nested-dissection leaf size in nodes (default 64)
 *   n_threads        host threads for sc_factor (0 = all cores)
 *   use_graph        1 = sc_assemble captures its kernel launches once into a
 *                    HIP graph and replays it on every later call (the plan's
 *                    buffers and tables are fixed, so the graph stays valid);
 *                    sc_apply_implicit captures its triangular sweeps once
 *                    (they touch plan-owned buffers only) and launches the
 *                    scatter of p and the gather into q eagerly around each
 *                    replay, so any p / q pointers reuse the one graph; calls
 *                    made while kernel timing is enabled launch eagerly
 *   assembly_kernels 0 = library default (two launches), 1 = overlapped:
 *                    the batch is cut into groups of subdomains and the SYRK
 *                    of group g runs on a second, library-owned stream while
 *                    the TRSM of group g+1 runs on the caller's stream (event
 *                    dependencies; the call returns with the caller's stream
 *                    waiting for the last SYRK), 2 = two launches (all TRSM
 *                    tiles, then all SYRK tiles)
 *   disable_reach    0 (default) = a TRSM column tile visits only the factor
 *                    blocks that hold rows on the elimination-tree paths of
 *                    its pivots: column j of X = L^{-1} P B^T is nonzero only
 *                    on the path from its pivot to the root, so every other
 *                    block works on zero rows (the result is the same up to
 *                    the sign of zeros); 1 = visit every block from the
 *                    tile's first pivot on (the staircase of Sec. 3.2 alone)
 *   block_split      GPU factor blocks (Sec. 3.2 factor splitting; the
 *                    non-uniform splitting of the Sec. 4.1 footnote): 0
 *                    (default) = uniform column ranges of panel_width
 *                    columns; 1 = ranges that
 *                    follow the supernodal elimination tree: a block is a
 *                    whole subtree or the top part of one (never two
 *                    unrelated subtrees), at most panel_width columns, so
 *                    that the blocks of disjoint subtrees are independent
 *                    (the implicit apply then solves them in parallel)
 *   select_iters     per-subdomain choice between the explicit and the
 *                    implicit approach (Sec. 5: the best approach depends on
 *                    the subdomain size and the iteration count): 0 (default)
 *                    = every subdomain explicit; k > 0 = the solver is
 *                    expected to apply the operator k times, and a subdomain
 *                    whose predicted amortisation point n* (sc_query_selection)
 *                    exceeds k is applied implicitly: sc_assemble skips it,
 *                    sc_apply and sc_pcpg apply it with the factor
 *                    (eq. (11)), the others with F (eq. (12)); the first
 *                    such call builds the implicit schedule and workspace
 *                    (device allocations, as sc_apply_implicit's first call
 *                    does).  The prediction: t_asm = structural flops /
 *                    select_model[0] TFLOP/s, t_expl = stored F bytes /
 *                    select_model[1] GB/s, t_impl = 16 nnz(L) /
 *                    select_model[2] GB/s (two FP64 sweeps), n* = t_asm /
 *                    (t_impl - t_expl) (infinite when t_impl <= t_expl);
 *                    zeros = rates measured on MI355X (assembly FP64 45.6 /
 *                    mixed 75.7 TFLOP/s, explicit apply 5800 GB/s, implicit
 *                    apply 3190 GB/s)
 *   tune_classes, ntune_classes  settings per size class from
 *                    sc_autotune_classes (see sc_tune_class_t), borrowed for
 *                    the sc_plan_create call
 *   lower_only_csr   0 (default) = kreg_rowptr / kreg_col hold both triangles
 *                    of K_reg; 1 = only the entries on and below the diagonal
 *                    (col <= row; SC_ERR_INVALID_ARG otherwise), and the
 *                    value arrays of sc_factor / sc_preprocess follow that
 *                    pattern
 *   syrk_kind        SYRK work items for every subdomain a tune class does
 *                    not cover: 0 (default) = by size (64 x 64 blocks up to
 *                    16384 rows FP64 / 6144 mixed, 128 x 128 tiles above),
 *                    1 = 64 x 64 blocks, 2 = 128 x 128 tiles
 *   disable_pair_merge  0 (default) = the TRSM updates the rows below two
 *                    consecutive factor blocks once for both where the
 *                    first's rows below are the second's rows followed by
 *                    the second's rows below (Sec. 3.2: fewer
 *                    read-modify-writes of X; the result is bit for bit the
 *                    same); 1 = one update per block
 *   arena_cap_bytes  0 (default) = X (the temporary of the assembly, Sec. 3.1)
 *                    resident for the whole batch; > 0 = temporary-memory
 *                    waves: the batch is cut into waves of subdomains whose X
 *                    slabs fit this many bytes (XCD-interleaved, largest
 *                    first), sc_assemble runs TRSM + SYRK wave after wave on
 *                    one X buffer of the largest wave's size.  sc_plan_create
 *                    returns SC_ERR_OOM when one subdomain's X alone exceeds
 *                    the cap (before touching the device), SC_ERR_UNSUPPORTED
 *                    with assembly_kernels = 1
 */
typedef struct {
    int32_t precision;
    int32_t disable_staircase;
    int32_t panel_width;
    int32_t relax_width;
    int32_t leaf_nodes;
    int32_t n_threads;
    int32_t use_graph;
    int32_t assembly_kernels;
    int32_t disable_reach;
    int32_t block_split;
    int32_t select_iters;
    float select_model[3];
    int64_t arena_cap_bytes;
    const struct sc_tune_class_s* tune_classes;
    int32_t ntune_classes;
    int32_t lower_only_csr;
    int32_t syrk_kind;
    int32_t disable_pair_merge;
} sc_options_t;

/*
 * One size class of the autotuner (sc_autotune_classes): the settings used
 * for every subdomain with n_lo <= n < n_hi.  Passed back to sc_plan_create
 * through sc_options_t::tune_classes / ntune_classes (borrowed for that call
 * only); a subdomain outside every class takes the plan-wide options.
 *   panel_width   GPU factor block width, 16..64 (0 = plan option)
 *   block_split   0 uniform, 1 elimination-tree ranges, -1 = plan option
 *   syrk_kind     SYRK work items: 0 = by size (64 x 64 blocks up to 16384
 *                 rows FP64 / 6144 mixed, 128 x 128 tiles above), 1 = 64 x
 *                 64 blocks, 2 = 128 x 128 tiles
 *   ms_per_sub    measured assembly time per subdomain of the class sample
 *                 with these settings (output; informational)
 */
typedef struct sc_tune_class_s {
    int32_t n_lo, n_hi;
    int32_t panel_width;
    int32_t block_split;
    int32_t syrk_kind;
    float ms_per_sub;
} sc_tune_class_t;

/* Initialisation stage (Sec. 2.2): ordering, symbolic factorisation, staircase
 * plan (Sec. 3, column pivots and stable sort), GPU block and tile lists, and
 * allocation of every persistent device buffer (factor values, X, F, tables)
 * on the current HIP device.  `stream` is used for the table uploads and the
 * one-time clear of F.  Errors: SC_ERR_INVALID_ARG (bad descriptor: index out
 * of range, sign not +-1, n <= 0 or n >= 2^27, perm not a permutation),
 * SC_ERR_OOM, SC_ERR_DEVICE. */
sc_status_t sc_plan_create(const sc_subdomain_desc_t* sd, int32_t nsub,
                           const sc_options_t* opt, void* stream, sc_plan_t* out);

/* Preprocessing, part 1: numeric Cholesky of every P K_reg P^T on the host
 * (FP64, threads over subdomains), then an asynchronous upload of the factor
 * values on `stream` (plus the FP32 copy used by SC_PREC_MIXED).
 *   kreg_vals   [nsub] host pointers to the CSR values of each K_reg, same
 *               pattern as at plan creation
 *   failed_sub, failed_col  optional out: on SC_ERR_NOT_SPD the subdomain and
 *               permuted column of the first non-positive pivot */
sc_status_t sc_factor(sc_plan_t plan, const double* const* kreg_vals, void* stream,
                      int32_t* failed_sub, int32_t* failed_col);

/* Preprocessing, part 2 (the hot path, Sec. 3): on `stream`, for every
 * subdomain, X = L^{-1} P B^T with the staircase TRSM (factor splitting with
 * pruned row lists, Sec. 3.2) and F = X^T X with the staircase SYRK (Sec. 3.3),
 * both restricted to the rows of X on the elimination-tree paths of the
 * pivots unless disable_reach is set.  F stays on the device in the sorted
 * column order, as the lower triangle of 128 x 128 tiles (F is symmetric;
 * its structurally zero 64 x 64 blocks and the padding past m are cleared
 * once by sc_plan_create and never written again); the permutation back to the multiplier
 * order (Sec. 3) is applied to the vectors by sc_apply / sc_pcpg and to the
 * matrix by sc_get_F.  Asynchronous.  SC_ERR_STATE before sc_factor. */
sc_status_t sc_assemble(sc_plan_t plan, void* stream);

/* Whole preprocessing stage in one call, pipelined (Sec. 4.4, the whole
 * assembly including the numerical factorisation and the extraction of the
 * factors, with CPU-GPU overlap once the first subdomains are factorised):
 * host threads factor the subdomains group by group (the batch is cut into
 * up to 8 groups, each holding part of every XCD's work list, largest
 * subdomains first); as soon as every subdomain of the next group is
 * factored and extracted, that group's factor values are copied to the
 * device (one asynchronous copy; the FP32 copy in mixed precision) and its
 * TRSM tiles and SYRK items are launched on `stream`, while the host goes on
 * with the next groups.  The result equals sc_factor followed by
 * sc_assemble bit for bit.  Returns when every group has been launched;
 * the assembly completes on `stream`.  Arguments and errors as sc_factor
 * (on SC_ERR_NOT_SPD no group after the failing one is launched and the plan
 * is left unfactored).  Not captured into a graph and not timed by
 * sc_set_timing. */
sc_status_t sc_preprocess(sc_plan_t plan, const double* const* kreg_vals, void* stream,
                          int32_t* failed_sub, int32_t* failed_col);

/* Solution stage, explicit apply (eq. (12)): q_i = F_i p_i for every
 * subdomain, on `stream`.  p_dev, q_dev: device FP64 vectors of length
 * sc_query(...)->dual total, concatenated per subdomain in the original
 * multiplier order (offsets from sc_query).  Every stored tile of F is read
 * once and applied with its transpose as well; sums in a fixed order (the
 * result is reproducible bit for bit).  FP32-stored F (mixed) is read as FP32
 * and accumulated in FP64.  SC_ERR_STATE before sc_assemble. */
sc_status_t sc_apply(sc_plan_t plan, const double* p_dev, double* q_dev, void* stream);

/* Explicit apply that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same result as sc_apply, bit for bit
 * (same kernels, same summation order), with the partial sums of the stored
 * tiles in a fixed device array of the library (32 MiB per GPU, held until
 * the process ends) instead of the plan's buffer.  The batch runs in chunks
 * of whole subdomains, one after the other on `stream`.  Limit: every
 * subdomain needs m <= 23040 (its ceil(m/128)(ceil(m/128)+1)/2 stored tiles
 * must fit the 16384 the array holds); SC_ERR_UNSUPPORTED otherwise, before
 * anything is launched.  All calls on one GPU share its array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  Arguments and other errors as sc_apply; the call
 * is not timed by sc_set_timing. */
sc_status_t sc_apply_noalloc(sc_plan_t plan, const double* p_dev, double* q_dev, void* stream);

/* Solution stage, implicit apply (eq. (11)): q_i = B_i P^T L^{-T} L^{-1} P B_i^T
 * p_i with two sparse triangular solves on the device, same vector layout as
 * sc_apply.  SC_ERR_STATE before sc_factor. */
sc_status_t sc_apply_implicit(sc_plan_t plan, const double* p_dev, double* q_dev, void* stream);

/* Solution stage: projected conjugate gradients (Sec. 2.1: the dual problem
 * (7), solved by PCPG, applying F once per iteration) on every subdomain's own
 * dual problem, e = 0, identity preconditioner, FP64 vectors and scalars, F
 * applied as in sc_apply (FP32-stored F read as FP32, accumulated in FP64):
 *   lambda_0 = 0, r_0 = d, w_0 = P r_0, p_0 = w_0, P = I - G (G^T G)^{-1} G^T,
 *   q = F p, alpha = (w.w)/(p.q), lambda += alpha p, r -= alpha q,
 *   w' = P r, beta = (w'.w')/(w.w), p = w' + beta p.
 * G_i = B_i R_i is formed by the library from the kernel basis:
 *   R_host      [nsub] host pointers, R_i is n_i x k_i column-major (original
 *               DOF numbering); k_host [nsub], 0 <= k_i <= 8, G_i^T G_i must be
 *               nonsingular (SC_ERR_INVALID_ARG otherwise)
 *   d_dev       device FP64 right-hand side, dual layout (see sc_apply)
 *   lambda_dev  device FP64 output, dual layout
 *   iters       number of iterations (>= 0)
 *   wnorm_hist  optional host array [(iters + 1) * nsub]: ||w_k|| of every
 *               subdomain after iteration k (row k)
 * A subdomain whose w or p.q reaches zero keeps its iterate.  Synchronises
 * `stream` when wnorm_hist is given.  SC_ERR_STATE before sc_assemble. */
sc_status_t sc_pcpg(sc_plan_t plan, const double* const* R_host, const int32_t* k_host,
                    const double* d_dev, double* lambda_dev, int32_t iters, double* wnorm_hist,
                    void* stream);

/* Copy F_i (m_i x m_i, column-major, leading dimension ld >= m_i, original
 * multiplier order: the stored tiles expanded and permuted back on the host)
 * to `out` (host memory when on_device == 0, else device memory), converted
 * to FP64.  Synchronises `stream`. */
sc_status_t sc_get_F(sc_plan_t plan, int32_t sub, double* out, int32_t ld, int32_t on_device,
                     void* stream);

/* Sizes and statistics of subdomain `sub` (any out pointer may be NULL):
 *   n, m, dual_offset (offset of its multipliers in the concatenated dual
 *   vectors), nnzL (exact structural nonzeros of L), useful_flops (staircase
 *   TRSM + SYRK flop count: sum_i a(i)(2c_i - 1) + a(i)(a(i) + 1), with a(i)
 *   the number of columns whose pivot is <= i and c_i = nnz(L[:, i])). */
sc_status_t sc_query(sc_plan_t plan, int32_t sub, int64_t* n, int64_t* m, int64_t* dual_offset,
                     int64_t* nnzL, double* useful_flops);

/* The per-subdomain choice of select_iters: *implicit = 1 when subdomain
 * `sub` is applied with the factor, 0 when assembled; the predicted times (ms)
 * of its assembly, of one explicit and of one implicit application, and its
 * amortisation point n* (+inf when the implicit application is not slower).
 * Any out pointer may be NULL. */
sc_status_t sc_query_selection(sc_plan_t plan, int32_t sub, int32_t* implicit, double* t_asm_ms,
                               double* t_expl_ms, double* t_impl_ms, double* n_star);

/* Plan-wide totals: number of subdomains, total dual length, useful TRSM and
 * SYRK flops (as in sc_query), the same counts without the staircase
 * ("orig"), the structural counts (the same sums with a(i) replaced by r(i),
 * the number of columns of X whose row i is structurally nonzero: pivots in
 * the elimination subtree of i; the flops the result needs at all), and the
 * device bytes held by the plan. */
sc_status_t sc_plan_stats(sc_plan_t plan, int32_t* nsub, int64_t* dual_total,
                          double* trsm_useful, double* syrk_useful, double* trsm_dense,
                          double* syrk_dense, double* trsm_reach, double* syrk_reach,
                          int64_t* device_bytes);

/* Kernel timing.  While enabled, sc_assemble and sc_apply record HIP events
 * on their stream around each kernel they launch; sc_kernel_times adds up the
 * elapsed milliseconds of every completed launch since the last reset
 * (synchronising on the recorded events):
 *   ms[0] staircase TRSM, ms[1] staircase SYRK + permute-back,
 *   ms[2] explicit apply (GEMV), ms[3] implicit apply,
 *   ms[4] assembly launched by groups (first TRSM to last SYRK:
 *         assembly_kernels 1, or temporary-memory waves);
 *   counts[k] = number of launches of kernel k summed into ms[k].
 * `reset` != 0 clears the sums after reading.  Arrays hold 5 entries. */
sc_status_t sc_set_timing(sc_plan_t plan, int32_t enable);
sc_status_t sc_kernel_times(sc_plan_t plan, double* ms, int64_t* counts, int32_t reset);

/* Autotuner for the factor block width (Sec. 4.1: the block size trades the
 * zeros skipped against the overhead of small blocks; the best value depends
 * on the hardware and the subdomain size).  Times sc_assemble for every
 * candidate width on up to `sample` subdomains of the batch, chosen evenly
 * over the batch sorted by n, on the current device and `stream`:
 *   sd, nsub, base    the batch and the options to tune (panel_width ignored)
 *   kreg_vals         [nsub] CSR values, as for sc_factor
 *   candidates[ncand] widths to try (each in [16, 64])
 *   reps              timed repetitions per candidate (>= 1)
 *   best_width        out: the fastest candidate
 *   times_ms          optional out [ncand]: mean ms per sc_assemble
 * Allocates and frees temporary plans.  Errors as sc_plan_create/sc_factor. */
sc_status_t sc_autotune(const sc_subdomain_desc_t* sd, int32_t nsub, const sc_options_t* base,
                        const double* const* kreg_vals, const int32_t* candidates, int32_t ncand,
                        int32_t sample, int32_t reps, void* stream, int32_t* best_width,
                        double* times_ms);

/* Autotuner over size classes (Sec. 4.1 and Table 1: the best block size
 * depends on the hardware and on the subdomain size).  The batch's
 * subdomains are grouped by n into classes [2^k, 2^(k+1)) (the first from 0,
 * the last open); for every class with subdomains, up to `sample` of them
 * (evenly over the class, by n) are planned, factored and assembled for each
 * candidate setting, and the fastest mean sc_assemble time wins, searched
 * coordinate by coordinate: block split (uniform, etree) at width 64, then
 * the width (32, 48, 64), then the SYRK work items (64 x 64 blocks, 128 x 128
 * tiles).  With `cache_path` (may be NULL) the results are kept in a text
 * file, one line per (device, precision, class): classes found there for this
 * device and precision are not timed again, new ones are appended.
 *   sd, nsub, base, kreg_vals   the batch and the options to tune, as for
 *                               sc_plan_create / sc_factor
 *   sample, reps                subdomains per class sample (>= 1), timed
 *                               repetitions per candidate (>= 1)
 *   classes[max_classes]        out: the tuned classes, increasing n
 *   nclasses                    out: how many
 * Allocates and frees temporary plans on the current device; errors as
 * sc_plan_create / sc_factor, SC_ERR_INVALID_ARG when max_classes is too small,
 * SC_ERR_DEVICE when the cache file cannot be written. */
sc_status_t sc_autotune_classes(const sc_subdomain_desc_t* sd, int32_t nsub, const sc_options_t* base,
                                const double* const* kreg_vals, int32_t sample, int32_t reps,
                                const char* cache_path, void* stream, sc_tune_class_t* classes,
                                int32_t max_classes, int32_t* nclasses);

/* Release every device and host buffer of the plan, after waiting for the
 * device (work queued on any stream may still use them).  NULL is accepted. */
sc_status_t sc_plan_destroy(sc_plan_t plan);

/* Thread-local message describing the last failure ("" if none). */
const char* sc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCASM_H */
