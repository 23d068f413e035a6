// Device-side tables shared by the kernels and the host code that builds them.
#pragma once
#include <cstdint>

namespace scasm {

// Width of a column tile of X (and of an F output tile): 4 stripes of 16
// columns, one stripe per wavefront in the TRSM.
constexpr int kTile = 64;
constexpr int kStripe = 16;
constexpr int kMaxPanel = 64;      // GPU panel width bound the TRSM kernel is built for
constexpr int kSyrkTile = 128;     // edge of an F output tile (two X column tiles)
constexpr int kFTileElems = kSyrkTile * kSyrkTile;
// Workgroups are dispatched to the accelerator's XCDs round-robin (workgroup
// k runs on XCD k mod kNumXcd); work lists are interleaved so that all items
// of one subdomain share an XCD and its L2.
constexpr int kNumXcd = 8;
// Overlapped assembly: the batch is cut into this many groups of subdomains
// (each XCD's list into consecutive parts); the SYRK of a group runs on a
// second stream while the TRSM of the next group runs.
constexpr int kOverlapGroups = 8;

struct SubDev {
    int32_t n, m, nblocks, ntiles;
    int64_t blk_off;     // first block in the global block table
    int64_t rows_off;    // first entry of this subdomain's row array
    int64_t lval_off;    // first factor value
    int64_t col_off;     // first entry of piv / pi / sign (sorted order)
    int64_t tile_off;    // first tile in the global tile table
    int64_t F_off;       // first element of F: packed lower tiles in sorted column order
    int64_t ftile_off;   // first stored F tile of this subdomain (apply partial sums)
    int64_t dual_off;    // offset of the subdomain's multipliers in dual vectors
};

// One column tile of X: sorted columns [64*tile, 64*tile + ncols) of subdomain
// `sub`.  Its slab holds rows [kstart, n) x 64 columns, row-major.
struct TileDev {
    int32_t sub, tile, kstart, ncols;
    int64_t x_off;
    int32_t start_block[4];   // first factor block each 16-column stripe works on
    int64_t visit_off;        // blocks the tile visits: visit[visit_off .. + nvisit),
    int32_t nvisit, pad;      // increasing indices relative to the subdomain's first block
};

// SYRK work item.  Subdomains with n <= kSyrkBlockMaxN (FP64; FP32:
// kSyrkBlockMaxNMixed): a 64 x 64 block of F
// (I >= J in units of 64-column X tiles), its k-range a list of 16-row steps
// (first rows at ksteps[step_off .. step_off + nsteps)) where both X tiles can
// hold a nonzero row.  Larger subdomains: a 128 x 128 tile of F (I >= J in
// units of kSyrkTile), each step entry = first row | slab bits <<
// kStepSlabShift, bit q set when 64-column slab q (2I, 2I+1, 2J, 2J+1) has a
// nonzero row in the step.  Every other step adds zero products.  Also used,
// in units of kSyrkTile and without steps, for the stored F tiles of the apply.
struct SyrkItem {
    int32_t sub;
    int32_t I, J;
    int32_t nsteps;
    int64_t step_off;
};
// measured on the elasticity batches: the FP64 blocks beat the tiles up to
// n = 14739 and lose at 27783; the FP32 tiles win above ~6000
constexpr int kSyrkBlockMaxN = 16384;
constexpr int kSyrkBlockMaxNMixed = 6144;
constexpr int kStepSlabShift = 27;
constexpr int kStepRowMask = (1 << kStepSlabShift) - 1;   // rows below 2^27 (checked at plan creation)

struct BlockDev {
    int32_t row0, w, nbelow;
    int32_t flags;       // bit 0: merged with the next block in the TRSM's updates below
    int64_t lval_off;    // diagonal block (w x w, column-major), relative to the subdomain's lval_off
    int64_t rows_off;    // relative to the subdomain's rows_off
    int64_t aoff;        // pruned rows as MFMA A tiles, relative to the subdomain's lval_off
    int64_t linv_off;    // inverse of the diagonal block as MFMA A tiles (same base)
};

}  // namespace scasm
