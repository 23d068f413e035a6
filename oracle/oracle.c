/*
 * ORACLE -- test infrastructure only.  Plain, slow CPU reference for the dual
 * Schur complement of one FETI subdomain.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark call it; the product library
 * never links or loads it, and it shares no code with the product library.
 *
 * What it computes (paper, Sec. 2.1 eq. (9) and Sec. 2.2 eq. (10)):
 *     F = B K_reg^{-1} B^T = Y^T Y,   Y = L^{-1} B^T,   L L^T = K_reg
 * (the SYRK form of Sec. 3.1, eq. (14)).  B^T has one entry sign_j in row
 * dof_j of column j.  Steps, in the paper's order and nothing more:
 *   1. Cholesky factor L of K_reg in the NATURAL order (no fill-reducing
 *      permutation: the permutation changes rounding only, never F), by the
 *      textbook row-by-row (Cholesky-Banachiewicz) recurrence
 *          L[i][j] = (K[i][j] - sum_{k<j} L[i][k] L[j][k]) / L[j][j]
 *          L[i][i] = sqrt(K[i][i] - sum_{k<i} L[i][k]^2).
 *      Row i of L has no entry left of the first nonzero of row i of K
 *      (envelope property), so each row is stored from that column on; the
 *      sums run over the columns both rows store, every other term being an
 *      exact zero.
 *   2. Y = L^{-1} B^T column by column, forward substitution over all rows
 *      (no skipping of the zeros above the pivot).
 *   3. F = Y^T Y, every entry of the lower triangle, mirrored.
 * Arithmetic: long double (x87, 64-bit significand) or double, chosen per
 * call; results are rounded to double on output.
 *
 * The `mutation` argument plants one deliberate mistake (tests use it to show
 * that the oracle's pins catch each plausible error); 0 = the correct oracle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* wall-clock seconds of the three steps of the last orc_schur call
 * (factorisation, forward substitution, Y^T Y); timing only */
static double g_phase[3];

static double wall_seconds(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

enum {
    MUT_NONE = 0,
    MUT_CHOL_SKIP_FIRST_TERM = 1,  /* Cholesky sum misses its first term */
    MUT_CHOL_PLUS = 2,             /* Cholesky update with + instead of - */
    MUT_CHOL_NO_SQRT = 3,          /* diagonal not square-rooted */
    MUT_FWD_NO_DIV = 4,            /* forward substitution forgets the diagonal */
    MUT_FWD_TRANSPOSED = 5,        /* solve with L^T (backward) instead of L */
    MUT_IGNORE_SIGN = 6,           /* B^T entries taken as +1 */
    MUT_SYRK_INDEX = 7,            /* F[a][b] = sum Y[k][a] Y[k][a] */
    MUT_DOF_OFF_BY_ONE = 8,        /* B^T entry placed at row dof+1 */
};

#define ORC_DEFINE(T, SUFFIX, SQRT)                                                    \
static int chol_##SUFFIX(int32_t n, const int64_t* rp, const int32_t* ci,               \
                         const double* v, const int64_t* start, const int32_t* first,  \
                         T* L, int mutation)                                           \
{                                                                                      \
    for (int32_t i = 0; i < n; ++i) {                                                  \
        T* Li = L + start[i] - first[i];          /* Li[j] = L[i][j] */                \
        for (int32_t j = first[i]; j <= i; ++j) Li[j] = 0;                             \
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)                                    \
            if (ci[p] <= i) Li[ci[p]] = (T)v[p];                                       \
        for (int32_t j = first[i]; j < i; ++j) {                                       \
            const T* Lj = L + start[j] - first[j];                                     \
            int32_t k0 = first[i] > first[j] ? first[i] : first[j];                    \
            if (mutation == MUT_CHOL_SKIP_FIRST_TERM && k0 < j) ++k0;                  \
            T s = Li[j];                                                               \
            for (int32_t k = k0; k < j; ++k) {                                         \
                if (mutation == MUT_CHOL_PLUS) s += Li[k] * Lj[k];                     \
                else s -= Li[k] * Lj[k];                                               \
            }                                                                          \
            Li[j] = s / Lj[j];                                                         \
        }                                                                              \
        T d = Li[i];                                                                   \
        for (int32_t k = first[i]; k < i; ++k) d -= Li[k] * Li[k];                     \
        if (!(d > 0)) return i + 1;                                                    \
        Li[i] = (mutation == MUT_CHOL_NO_SQRT) ? d : SQRT(d);                          \
    }                                                                                  \
    return 0;                                                                          \
}                                                                                      \
                                                                                       \
/* y <- L^{-1} y over all rows (or L^{-T} y for the planted transposition). */         \
static void fwd_##SUFFIX(int32_t n, const int64_t* start, const int32_t* first,         \
                         const T* L, T* y, int mutation)                               \
{                                                                                      \
    if (mutation == MUT_FWD_TRANSPOSED) {                                              \
        for (int32_t i = n - 1; i >= 0; --i) {                                         \
            const T* Li = L + start[i] - first[i];                                     \
            y[i] /= Li[i];                                                             \
            for (int32_t k = first[i]; k < i; ++k) y[k] -= Li[k] * y[i];               \
        }                                                                              \
        return;                                                                        \
    }                                                                                  \
    for (int32_t i = 0; i < n; ++i) {                                                  \
        const T* Li = L + start[i] - first[i];                                         \
        T s = y[i];                                                                    \
        for (int32_t k = first[i]; k < i; ++k) s -= Li[k] * y[k];                      \
        y[i] = (mutation == MUT_FWD_NO_DIV) ? s : s / Li[i];                           \
    }                                                                                  \
}                                                                                      \
                                                                                       \
static int schur_##SUFFIX(int32_t n, const int64_t* rp, const int32_t* ci,              \
                          const double* v, int32_t m, const int32_t* dof,              \
                          const int8_t* sign, int32_t nsel, const int32_t* sel,        \
                          double* F, double* Yout, int nthreads, int mutation)         \
{                                                                                      \
    int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));      \
    int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));              \
    if (!first || !start) { free(first); free(start); return -2; }                     \
    start[0] = 0;                                                                      \
    for (int32_t i = 0; i < n; ++i) {                                                  \
        int32_t f = i;                                                                 \
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) if (ci[p] < f) f = ci[p];          \
        first[i] = f;                                                                  \
        start[i + 1] = start[i] + (i - f + 1);                                         \
    }                                                                                  \
    T* L = (T*)malloc(sizeof(T) * (size_t)(start[n] > 0 ? start[n] : 1));              \
    T* Y = (T*)calloc((size_t)n * (size_t)(nsel > 0 ? nsel : 1), sizeof(T));           \
    if (!L || !Y) { free(first); free(start); free(L); free(Y); return -2; }           \
    double t0 = wall_seconds();                                                        \
    int bad = chol_##SUFFIX(n, rp, ci, v, start, first, L, mutation);                  \
    if (bad) { free(first); free(start); free(L); free(Y); return bad; }               \
    double t1 = wall_seconds();                                                        \
    (void)nthreads;                                                                    \
    _Pragma("omp parallel for schedule(dynamic, 4) num_threads(nthreads)")             \
    for (int32_t s = 0; s < nsel; ++s) {                                               \
        int32_t j = sel ? sel[s] : s;                                                  \
        T* y = Y + (size_t)s * (size_t)n;                                              \
        int32_t row = dof[j] + (mutation == MUT_DOF_OFF_BY_ONE ? 1 : 0);               \
        if (row >= n) row = n - 1;                                                     \
        y[row] = (mutation == MUT_IGNORE_SIGN) ? (T)1 : (T)sign[j];                    \
        fwd_##SUFFIX(n, start, first, L, y, mutation);                                 \
    }                                                                                  \
    double t2 = wall_seconds();                                                        \
    _Pragma("omp parallel for schedule(dynamic, 4) num_threads(nthreads)")             \
    for (int32_t b = 0; b < nsel; ++b) {                                               \
        const T* yb = Y + (size_t)b * (size_t)n;                                       \
        for (int32_t a = b; a < nsel; ++a) {                                           \
            const T* ya = Y + (size_t)a * (size_t)n;                                   \
            const T* yb2 = (mutation == MUT_SYRK_INDEX) ? ya : yb;                     \
            T s = 0;                                                                   \
            for (int32_t k = 0; k < n; ++k) s += ya[k] * yb2[k];                       \
            F[(size_t)b * nsel + a] = (double)s;                                       \
            F[(size_t)a * nsel + b] = (double)s;                                       \
        }                                                                              \
    }                                                                                  \
    g_phase[0] = t1 - t0;                                                              \
    g_phase[1] = t2 - t1;                                                              \
    g_phase[2] = wall_seconds() - t2;                                                  \
    if (Yout)                                                                          \
        for (size_t t = 0; t < (size_t)n * (size_t)nsel; ++t) Yout[t] = (double)Y[t];  \
    free(first); free(start); free(L); free(Y);                                        \
    return 0;                                                                          \
}

ORC_DEFINE(long double, ld, sqrtl)
ORC_DEFINE(double, d, sqrt)

/*
 * F[S,S] of B K_reg^{-1} B^T for the column subset S (sel[0..nsel), or all m
 * columns when sel == NULL, nsel == m).
 *   n, rowptr[n+1], col, val : K_reg in CSR, both triangles (only the lower
 *                              triangle is read), int64 row pointers
 *   m, dof[m], sign[m]       : B^T, one entry sign[j] (+1/-1) in row dof[j]
 *   prec                     : 1 = long double, 0 = double
 *   F                        : out, nsel*nsel, column-major (symmetric)
 *   Y                        : optional out, n*nsel column-major = L^{-1} B^T[:,S]
 * Returns 0; i+1 when pivot i of the Cholesky factor is not positive; -1 on a
 * bad argument; -2 when memory runs out.
 */
int orc_schur(int32_t n, const int64_t* rowptr, const int32_t* col, const double* val,
              int32_t m, const int32_t* dof, const int8_t* sign, int32_t nsel,
              const int32_t* sel, int32_t prec, double* F, double* Y, int32_t nthreads,
              int32_t mutation)
{
    if (n <= 0 || m < 0 || nsel < 0 || !rowptr || !col || !val || !F) return -1;
    if (nsel > 0 && (!dof || !sign)) return -1;
    if (!sel && nsel != m) return -1;
    for (int32_t s = 0; s < nsel; ++s) {
        int32_t j = sel ? sel[s] : s;
        if (j < 0 || j >= m || dof[j] < 0 || dof[j] >= n) return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if (prec == 1)
        return schur_ld(n, rowptr, col, val, m, dof, sign, nsel, sel, F, Y, nthreads, mutation);
    return schur_d(n, rowptr, col, val, m, dof, sign, nsel, sel, F, Y, nthreads, mutation);
}

/* Seconds spent by the last orc_schur call in its three steps: out[0]
 * Cholesky, out[1] forward substitution, out[2] Y^T Y. */
void orc_last_phase_seconds(double* out)
{
    out[0] = g_phase[0];
    out[1] = g_phase[1];
    out[2] = g_phase[2];
}

/* Cholesky factor alone (long double), returned densely (n*n, row-major, upper
 * part zero) for small-size tests.  Returns as orc_schur. */
int orc_cholesky_dense(int32_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                       double* Lout)
{
    if (n <= 0 || !Lout) return -1;
    int32_t* first = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    start[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t f = i;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) if (col[p] < f) f = col[p];
        first[i] = f;
        start[i + 1] = start[i] + (i - f + 1);
    }
    long double* L = (long double*)malloc(sizeof(long double) * (size_t)start[n]);
    int bad = chol_ld(n, rowptr, col, val, start, first, L, 0);
    if (!bad) {
        memset(Lout, 0, sizeof(double) * (size_t)n * (size_t)n);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t j = first[i]; j <= i; ++j)
                Lout[(size_t)i * n + j] = (double)L[start[i] + j - first[i]];
    }
    free(first); free(start); free(L);
    return bad;
}
