// Host-side logic of the library that needs no GPU: the octree leaves of the
// block-diagonal preconditioner and the work plans of the pairwise and banded
// pair sweeps.  Plain C++17 (no HIP), so that a host build with sanitizers
// tests it on the CPU.  Internal; not part of the public ABI.
#pragma once

#include <cstdint>
#include <vector>

namespace pbk {

constexpr int TILE = 256;   // points per tile of the pair sweeps (staged in LDS per step)

// The hardware hands the workgroups of a launch to the XCDs in turn
// (workgroup b to XCD b mod XCDS); each XCD has its own L2.
constexpr int XCDS = 8;

// Work items of the pairwise sweeps (4 int32 each: I, J0, J1, slot): target
// tile I against source tiles J0..J1-1 (J0 >= I; the tile J = I runs forward
// only); slot is the item's row record, and row_start[K]..row_start[K+1] are
// the slots of target tile K, in ascending J0.  Every tile pair I <= J < T
// belongs to exactly one item.  From SYM_STRIP_MIN_TILES tiles on, the source
// tiles are cut into 2 XCDS strips of equal width and no item crosses a strip
// boundary; strips k and
// 2 XCDS - 1 - k (equal numbers of tile pairs between them) belong to XCD k,
// and the items are ordered so that launch position b holds an item of XCD
// b mod XCDS, longest first on each XCD.  Each XCD then streams an eighth of
// the sources through its L2.  About target_blocks items.
constexpr int SYM_STRIP_MIN_TILES = 512;
struct SymPlan {
    int64_t npad = 0;
    int n_tiles = 0;      // T = npad / TILE
    int tiles_per_item = 0;
    int n_items = 0;
    int strips = 1;       // 2 XCDS, or 1 below SYM_STRIP_MIN_TILES tiles
};
SymPlan plan_sym(int64_t npad, int target_blocks, std::vector<int32_t> &items,
                 std::vector<int32_t> &row_start);

// Banded pairwise sweep (pb_kernels.h, sweep kind PB_SWEEP_BANDED): a block
// of BAND_WAVES waves holds BAND_MT target tiles (a macro tile); a work item
// is a band of macro tiles [m0, m1) against a run of source tiles [j0, j1),
// j0 at or after the band's first tile.  Its records (2 x TILE floats each)
// hold the rows of each target tile I of the band over the run (slot
// rslot + I - BAND_MT m0, written when j1 > I) and the column sums of each
// source tile J of the run over the band (slot cslot + J - j0).
constexpr int BAND_WAVES = 8;
constexpr int BAND_MT = 2 * BAND_WAVES * 64 / TILE;   // target tiles per macro tile (4)
constexpr int BAND_RUN_MAX = 24;                      // source tiles per item (LDS)
struct BandItem {
    int32_t m0, m1, j0, j1, rslot, cslot, pad0, pad1;
};
struct BandPlan {
    int64_t npad = 0;
    int n_tiles = 0, n_items = 0, run = 0, band = 0, target = 0;
    int64_t n_records = 0;
};
// Items for npad points (npad / TILE tiles), about target_items of them,
// longest first; rec_start[K]..rec_start[K+1] of rec_idx list the records of
// tile K's rows: its row records in run order, then its column records in
// band order.  Every unordered tile pair (I <= J) belongs to exactly one item.
BandPlan plan_band(int64_t npad, int target_items, std::vector<BandItem> &items,
                   std::vector<int32_t> &rec_start, std::vector<int32_t> &rec_idx);

// Octree leaves of n points (Sec. 2.2.3's tree, used for the leaf blocks of
// Sec. 2.2.4): a cell with more than n0 points is split at its centre into
// octants (stable), a cell with at most n0 points is a leaf; perm lists the
// points leaf by leaf in depth-first octant order and start[l] .. start[l + 1]
// delimits leaf l.  With `threads`, the subtrees of the root's children are
// built on their own threads; the result does not depend on it.
void build_leaves(const double *x, const double *y, const double *z, int64_t n, int n0,
                  std::vector<int32_t> &perm, std::vector<int32_t> &start, bool threads = true);

}  // namespace pbk
