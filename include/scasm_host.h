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

#ifdef __cplusplus
}
#endif

#endif /* SCASM_HOST_H */
