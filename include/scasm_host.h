/*
 * scasm -- host-only introspection of the planner (no HIP device needed).
 *
 * Runs the initialisation stage (ordering, symbolic factorisation, staircase
 * plan) and, when values are given, the numeric factorisation of one
 * subdomain on the host, and reports what the device path would receive.
 * Used to test the planner on machines without a GPU.
 */
#ifndef SCASM_HOST_H
#define SCASM_HOST_H

#include <stdint.h>

#include "scasm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t n, m;
    int64_t nnzL;          /* exact structural nonzeros of L (incl. diagonal) */
    int64_t nnzL_stored;   /* supernodal storage incl. explicit zeros          */
    int64_t nsuper;        /* supernodes after relaxed amalgamation            */
    int64_t nblocks;       /* GPU factor blocks (panels)                       */
    int64_t max_width;     /* widest supernode                                 */
    int64_t sum_below;     /* sum over blocks of pruned rows below the block   */
    double trsm_useful, syrk_useful;   /* staircase flop counts (Sec. 3.2-3.3) */
    double trsm_dense, syrk_dense;     /* same factor without the staircase    */
    double factor_flops;               /* sum_j c_j^2 (estimate)               */
    int64_t trsm_visits;   /* (column tile, factor block) pairs the TRSM visits */
    int64_t stair_visits;  /* the same with the staircase alone (no reach)      */
    double trsm_reach, syrk_reach;     /* structural counts: a(i) replaced by
                                          r(i) = columns of X nonzero in row i */
    double t_asm_ms, t_expl_ms, t_impl_ms, n_star;   /* the select_iters
                                          prediction (sc_options_t) */
    int64_t merge_pairs;   /* factor block pairs whose TRSM updates below merge
                              (0 with disable_pair_merge)                 */
    int64_t merged_rows;   /* pruned-row updates the merging saves: over the
                              column tiles, the second block's pruned rows
                              for every visit of a pair's first block that
                              the second follows                          */
    int64_t pruned_updates;  /* pruned-row updates of the TRSM without merging:
                              over the column tiles, the pruned rows of every
                              visited block                                */
} sc_host_info_t;

/*
 * sd, opt        as for sc_plan_create (one subdomain)
 * kreg_vals      optional CSR values of K_reg; when given, L is computed
 * perm_out       optional [n]: fill-reducing order, perm[new] = old
 * L_out          optional [n*n] row-major dense copy of L (small n only;
 *                requires kreg_vals)
 * piv_out, pi_out optional [m]: pivots in sorted order, sorted -> original
 * info           optional statistics
 * Returns SC_OK, SC_ERR_INVALID_ARG (bad descriptor or n > 4096 with L_out),
 * SC_ERR_NOT_SPD (with *failed_col set when failed_col is not NULL).
 */
sc_status_t sc_host_analyze(const sc_subdomain_desc_t* sd, const sc_options_t* opt,
                            const double* kreg_vals, int32_t* perm_out, double* L_out,
                            int32_t* piv_out, int32_t* pi_out, sc_host_info_t* info,
                            int32_t* failed_col);

/*
 * The factor blocks the staircase TRSM visits for each 64-column tile of X
 * (columns in the sorted order of sc_host_analyze's piv_out), and the 16-row
 * steps in which each tile can hold nonzero rows (the SYRK's k-steps are the
 * steps marked for both of its tiles), as the device path receives them.
 *   sd, opt      as for sc_host_analyze
 *   counts       [4] out: number of blocks, number of tiles, total visits,
 *                mask words per tile
 *   block_row0   optional [blocks + 1] out: first row of each block, then n
 *   visit_ptr    optional [tiles + 1] out: tile t visits
 *                visit[visit_ptr[t] .. visit_ptr[t + 1])
 *   visit        optional [capacity] out: block indices, increasing per tile
 *   step_mask    optional [tiles * words] out: bit q of word q / 64 of tile t
 *                set when rows [16 q, 16 q + 16) can hold nonzeros of tile t
 * Call once with the optional outputs NULL to size them.  Returns SC_OK, or
 * SC_ERR_INVALID_ARG for a bad descriptor or when capacity < total visits
 * with visit given (counts are filled in either case).
 */
sc_status_t sc_host_tile_visits(const sc_subdomain_desc_t* sd, const sc_options_t* opt, int64_t* counts,
                                int32_t* block_row0, int64_t* visit_ptr, int32_t* visit, int64_t capacity,
                                uint64_t* step_mask);

#ifdef __cplusplus
}
#endif

#endif /* SCASM_HOST_H */
