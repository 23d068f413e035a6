// Host planner: ordering, symbolic and numeric sparse Cholesky, staircase plan.
//
// The factor L of the permuted regularised stiffness P K_reg P^T (paper,
// Sec. 2.2 eq. (10) and the two-stage factorisation it describes) is held in
// supernodal form: supernode s owns the contiguous permuted columns
// [first_s, first_s + w_s) and a sorted row list whose first w_s entries are
// its own columns and whose remaining r_s entries are the rows below it; the
// values are a dense column-major panel of (w_s + r_s) x w_s doubles.
//
// The staircase plan follows Sec. 3: the pivot of multiplier column j is
// p_j = iperm[dof_j]; columns are stably sorted by (p_j, j) so that pivots
// descend left to right (the "stepped" shape), and the solution X = L^{-1}
// P B^T is zero above each pivot.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace scasm {

struct SubdomainInput {
    int32_t n = 0;
    const int64_t* rowptr = nullptr;   // K_reg CSR (both triangles), n+1
    const int32_t* col = nullptr;
    int32_t m = 0;
    const int32_t* dof = nullptr;      // [m]
    const int8_t* sign = nullptr;      // [m]
    const int32_t* perm = nullptr;     // optional [n], new -> old
    const double* coords = nullptr;    // optional [n / dofs_per_node][dim]
    int32_t dim = 0;
    int32_t dofs_per_node = 1;
};

struct PlanOptions {
    int32_t leaf_nodes = 64;          // nested-dissection leaf size (nodes)
    int32_t relax_width = 64;         // relaxed amalgamation merges up to this width
    double relax_zero_frac = 0.5;     // ... if the merged zero fraction stays below this
    int32_t panel_width = 64;         // GPU factor block width (uniform blocks)
    int32_t staircase = 1;            // 0 = every column treated as pivot 0 ("orig")
    int32_t reach = 1;                // 0 = a TRSM tile sweeps every block after its first pivot's
    int32_t block_split = 0;          // 0 = uniform column ranges of panel_width; 1 = ranges that
                                      // follow the supernodal elimination tree (a block is a subtree
                                      // or the top part of one, at most panel_width columns)
};

// One GPU factor block (Sec. 3.2, factor splitting with pruning): the column
// range [row0, row0 + w) of L (uniform width except the last, or following the
// elimination tree: PlanOptions::block_split).  Its values:
//   * the dense diagonal triangle, w x w column-major (leading dimension
//     ld = w) at lval_off;
//   * the `nbelow` non-empty rows of L[row0 + w :, block] (pruning), whose
//     global indices start at rows_off in the block row array, stored at aoff
//     as MFMA A-operand tiles: rows in tiles of 16, columns in slices of 4;
//     tile (rt, ks) holds 64 values at aoff + 64 (rt * nks + ks), value
//     (row 16 rt + i, column 4 ks + k) at position i + 16 k, nks = ceil(w/4),
//     zero padded;
//   * the inverse of the diagonal triangle (lower triangular) at linv_off, in
//     the same tile format, only the tiles on or below the diagonal: row
//     tile rt holds k-slices ks < min(nks, 4 (rt + 1)), tile (rt, ks) at
//     linv_off + 64 (2 rt (rt + 1) + ks).
struct BlockDesc {
    int32_t row0;
    int32_t w;
    int32_t nbelow;
    int32_t ld;
    int64_t lval_off;
    int64_t rows_off;
    int64_t aoff;
    int64_t linv_off;
};

struct SubPlan {
    int32_t n = 0, m = 0, dpn = 1;
    std::vector<int32_t> perm, iperm;          // perm[new] = old
    std::vector<int32_t> parent;               // column elimination tree
    std::vector<int32_t> colcount;             // exact nnz(L[:, j]) incl. diagonal
    // supernodes
    int32_t nsuper = 0;
    std::vector<int32_t> sfirst;               // nsuper + 1
    std::vector<int64_t> srow_ptr;             // nsuper + 1
    std::vector<int32_t> srows;                // own columns then rows below
    std::vector<int64_t> spanel_off;           // nsuper + 1, doubles
    int64_t nval = 0;
    std::vector<int32_t> col2super;
    std::vector<int64_t> kmap;                 // CSR entry -> panel slot, -1 = upper part
    std::vector<int32_t> dof;                  // [m] B^T columns as given (original order)
    std::vector<int8_t> sign;                  // [m]
    // staircase
    std::vector<int32_t> piv;                  // [m] pivots in sorted order
    std::vector<int32_t> pi;                   // [m] sorted position -> original column
    std::vector<int8_t> sign_sorted;           // [m]
    std::vector<int32_t> active;               // a(i) for i in [0, n)
    // GPU blocks
    int32_t block_width = 64;
    std::vector<BlockDesc> blocks;
    std::vector<int32_t> brows;                // pruned rows of every block (lists start 16-byte aligned)
    int64_t bval = 0;                          // values in all block panels
    std::vector<int32_t> block_of_row;         // row -> block index
    // blocks each 64-column tile of X visits (increasing): tile t holds
    // visit[visit_ptr[t] .. visit_ptr[t + 1])
    std::vector<int64_t> visit_ptr;
    std::vector<int32_t> visit;
    std::vector<uint64_t> visit_rows;          // per visit: rows of the block on the paths (bit i = row0 + i)
    int64_t visits_stair = 0;                  // the same count for the staircase alone
    // 16-row steps holding nonzero rows of each 64-column tile of X (bit q of
    // word q / 64 = rows [16 q, 16 q + 16)), mask_words words per tile
    int32_t mask_words = 0;
    std::vector<uint64_t> step_mask;
    // statistics
    int64_t nnzL = 0;                          // exact
    int64_t nnzL_stored = 0;                   // supernodal storage incl. explicit zeros
    double trsm_useful = 0, syrk_useful = 0;   // element-granular staircase counts
    double trsm_dense = 0, syrk_dense = 0;     // same factor, no staircase ("orig")
    double trsm_reach = 0, syrk_reach = 0;     // structural counts: only the nonzero rows of X
    double factor_flops = 0;
};

// Returns "" on success, else an error message; `code` receives 1 for a bad
// argument.
std::string build_plan(const SubdomainInput& in, const PlanOptions& opt, SubPlan& out, int& code);

// Numeric supernodal Cholesky into `vals` (plan.nval doubles).  Returns -1 on
// success, else the permuted column whose pivot is not positive.
int64_t factor_numeric(const SubPlan& plan, const double* kvals, double* vals);

// Copies the supernodal factor values into the GPU block panels (plan.bval
// doubles): the extraction of the dense diagonal blocks and of the non-empty
// sub-diagonal rows.
void repack_blocks(const SubPlan& plan, const double* vals, double* bvals);

// Blocks whose update of the rows below the TRSM merges with the next
// block's (flag 1 per block): b + 1 a whole number of 16-row tiles wide and
// the pruned rows of b exactly the rows of b + 1 followed by the pruned rows
// of b + 1 (the panels of one supernode, or a child whose structure is its
// parent's); paired greedily from the first block, so a block is in at most
// one pair.
std::vector<int32_t> merge_pairs(const SubPlan& plan);

}  // namespace scasm
