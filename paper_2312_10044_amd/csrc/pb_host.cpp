// Host-side logic of the library (see pb_host.h): the preconditioner's
// octree leaves and the work plan of the banded pair sweep.  Plain C++17, compiled into the library by the host compiler
// and, for the tests, by g++ with sanitizers.
#include "pb_host.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <system_error>
#include <thread>
#include <vector>

namespace pbk {

// Leaves of the octree over the collocation points (Sec. 2.2.3): the root is
// the cube around the bounding box of the points; a cluster with more than n0
// points splits into its eight child cubes (octant = (x >= cx) + 2 (y >= cy)
// + 4 (z >= cz), child centres c +- h/2), empty children are dropped, leaves
// are listed depth first in octant order, points in increasing index order.
// The tree is built in place: each cluster is one range of `perm`, split by a
// stable counting sort into its octants, so the ranges of the children follow
// each other in octant order and the final `perm` lists the leaves depth
// first.
namespace {

struct LeafFrame {
    int64_t a, b;   // range of perm
    double c[3], h;
    int depth;
};

// Splits frame f of perm by octant (stable) and returns the child frames in
// octant order; or, if f is a leaf, appends its leaf ends to `ends`.
void split_frame(const double *x, const double *y, const double *z, int n0, const LeafFrame &f,
                 int32_t *perm, int32_t *tmp, uint8_t *oct, std::vector<LeafFrame> &kids,
                 std::vector<int32_t> &ends)
{
    kids.clear();
    const int64_t m = f.b - f.a;
    if (m <= n0 || f.depth >= 40) {
        // at the depth limit (coincident points) the leaf is cut into
        // consecutive runs of at most n0 points
        for (int64_t a = f.a; a < f.b; a += n0)
            ends.push_back((int32_t)std::min(f.b, a + (int64_t)n0));
        return;
    }
    int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t k = f.a; k < f.b; ++k) {
        const int32_t i = perm[k];
        const int o =
            (x[i] >= f.c[0] ? 1 : 0) + (y[i] >= f.c[1] ? 2 : 0) + (z[i] >= f.c[2] ? 4 : 0);
        oct[k] = (uint8_t)o;
        ++cnt[o];
    }
    int64_t off[9];
    off[0] = f.a;
    for (int o = 0; o < 8; ++o)
        off[o + 1] = off[o] + cnt[o];
    int64_t put[8];
    for (int o = 0; o < 8; ++o)
        put[o] = off[o];
    for (int64_t k = f.a; k < f.b; ++k)
        tmp[put[oct[k]]++] = perm[k];
    std::copy(tmp + f.a, tmp + f.b, perm + f.a);
    const double hh = 0.5 * f.h;
    for (int o = 0; o < 8; ++o) {
        if (cnt[o] == 0)
            continue;
        kids.push_back(LeafFrame{off[o], off[o + 1],
                                 {f.c[0] + ((o & 1) ? hh : -hh), f.c[1] + ((o & 2) ? hh : -hh),
                                  f.c[2] + ((o & 4) ? hh : -hh)},
                                 hh, f.depth + 1});
    }
}

// Depth-first build of the subtree of `root`; leaf ends in octant order.
void build_subtree(const double *x, const double *y, const double *z, int n0,
                   const LeafFrame &root, int32_t *perm, int32_t *tmp, uint8_t *oct,
                   std::vector<int32_t> &ends)
{
    std::vector<LeafFrame> stack{root}, kids;
    while (!stack.empty()) {
        const LeafFrame f = stack.back();
        stack.pop_back();
        split_frame(x, y, z, n0, f, perm, tmp, oct, kids, ends);
        // children pushed in reverse so they pop in octant order
        for (auto it = kids.rbegin(); it != kids.rend(); ++it)
            stack.push_back(*it);
    }
}

}  // namespace

// Octree over the collocation points: a cell with more than n0 points is split
// at its centre into octants (stable), a cell with at most n0 points is a leaf;
// perm lists the points leaf by leaf in depth-first octant order and
// start[l] .. start[l + 1] delimits leaf l.  With `threads`, the subtrees of
// the root's children are built on their own threads (disjoint ranges of
// perm); the result does not depend on it.
void build_leaves(const double *x, const double *y, const double *z, int64_t n, int n0,
                  std::vector<int32_t> &perm, std::vector<int32_t> &start, bool threads)
{
    double lo[3] = {x[0], y[0], z[0]}, hi[3] = {x[0], y[0], z[0]};
    for (int64_t i = 1; i < n; ++i) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    perm.resize(n);
    for (int64_t i = 0; i < n; ++i)
        perm[i] = (int32_t)i;
    std::vector<int32_t> tmp(n);
    std::vector<uint8_t> oct(n);
    LeafFrame root{0, n, {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])},
                   0.0, 0};
    for (int k = 0; k < 3; ++k)
        root.h = std::max(root.h, 0.5 * (hi[k] - lo[k]));
    start.assign(1, 0);
    std::vector<LeafFrame> kids;
    std::vector<int32_t> ends;
    split_frame(x, y, z, n0, root, perm.data(), tmp.data(), oct.data(), kids, ends);
    if (kids.empty()) {
        start.insert(start.end(), ends.begin(), ends.end());
        return;
    }
    std::vector<std::vector<int32_t>> sub(kids.size());
    const bool threaded = threads && n >= 16384;
    std::vector<std::thread> pool;
    for (size_t k = 0; k < kids.size(); ++k) {
        auto job = [&, k] {
            build_subtree(x, y, z, n0, kids[k], perm.data(), tmp.data(), oct.data(), sub[k]);
        };
        bool spawned = false;
        if (threaded) {
            try {
                pool.emplace_back(job);
                spawned = true;
            } catch (const std::system_error &) {
                // no thread available: build this subtree here
            }
        }
        if (!spawned)
            job();
    }
    for (auto &t : pool)
        t.join();
    for (const auto &s : sub)
        start.insert(start.end(), s.begin(), s.end());
}

SymPlan plan_sym(int64_t npad, int target_blocks, std::vector<int32_t> &items,
                 std::vector<int32_t> &row_start)
{
    SymPlan pl;
    pl.npad = npad;
    const int T = (int)(npad / TILE);
    pl.n_tiles = T;
    const int64_t work = (int64_t)T * (T + 1) / 2;   // tile pairs incl. the diagonal
    const int64_t want = std::max(1, target_blocks);
    const int L = (int)std::max<int64_t>(1, (work + want - 1) / want);
    pl.tiles_per_item = L;
    // strips only where the source stream is well past an XCD's 4 MB L2 (12 KB
    // per FP32 tile, 16 KB per FP64 tile: 6 and 8 MB at 512 tiles); at 320
    // tiles (81,920 points) the unsplit runs measured faster
    const int NS = T >= SYM_STRIP_MIN_TILES ? 2 * XCDS : 1;
    pl.strips = NS;
    std::vector<int> edge(NS + 1);
    for (int k = 0; k <= NS; ++k)
        edge[k] = (int)((int64_t)k * T / NS);
    struct Row {
        int32_t I, j0, j1, slot;
        int xcd;
    };
    std::vector<Row> rows;
    row_start.assign(T + 1, 0);
    int slot = 0;
    for (int I = 0; I < T; ++I) {
        row_start[I] = slot;
        for (int k = 0; k < NS; ++k) {
            const int a = std::max(I, edge[k]), e = edge[k + 1];
            if (a >= e)
                continue;
            // the strip's part of the row in runs of at most L, of near-equal length
            const int len = e - a, nr = (len + L - 1) / L;
            for (int r = 0; r < nr; ++r) {
                const int j0 = a + (int)((int64_t)r * len / nr);
                const int j1 = a + (int)((int64_t)(r + 1) * len / nr);
                rows.push_back({I, j0, j1, slot++, NS == 1 ? 0 : (k < XCDS ? k : NS - 1 - k)});
            }
        }
    }
    row_start[T] = slot;
    pl.n_items = slot;
    // per XCD, longest first (stable: ascending I, then J0, among equals)
    std::vector<std::vector<int>> per(XCDS);
    for (int k = 0; k < slot; ++k)
        per[rows[k].xcd].push_back(k);
    for (auto &v : per)
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
            return rows[a].j1 - rows[a].j0 > rows[b].j1 - rows[b].j0;
        });
    items.clear();
    items.reserve(4 * (size_t)slot);
    size_t longest = 0;
    for (const auto &v : per)
        longest = std::max(longest, v.size());
    for (size_t q = 0; q < longest; ++q)
        for (int x = 0; x < XCDS; ++x)
            if (q < per[x].size()) {
                const Row &r = rows[per[x][q]];
                items.insert(items.end(), {r.I, r.j0, r.j1, r.slot});
            }
    return pl;
}

BandPlan plan_band(int64_t npad, int target_items, std::vector<BandItem> &items,
                   std::vector<int32_t> &rec_start, std::vector<int32_t> &rec_idx)
{
    BandPlan pl;
    pl.npad = npad;
    pl.target = target_items;
    const int T = (int)(npad / TILE);
    pl.n_tiles = T;
    const int n_macro = (T + BAND_MT - 1) / BAND_MT;
    // an item of `band` macro tiles and `run` source tiles covers about
    // BAND_MT band run tile pairs; aim at target_items items of the
    // T (T + 1) / 2 tile pairs, with runs and bands of about equal extent
    const double work = 0.5 * (double)T * (double)(T + 1);
    const double per_item = std::max(1.0, work / std::max(1, target_items));
    int run = (int)std::lround(std::sqrt(per_item));
    run = std::min(BAND_RUN_MAX, std::max(2, run));
    int band = (int)std::lround(per_item / (double)(BAND_MT * run));
    band = std::max(1, std::min(band, n_macro));
    pl.run = run;
    pl.band = band;
    struct Rec {
        BandItem it;
        int64_t work;
    };
    std::vector<Rec> all;
    int64_t slot = 0;
    // records of each tile K: rows (runs of its band reaching K), then
    // columns (items whose run holds K and whose band starts below K)
    std::vector<std::vector<int32_t>> rows(T), cols(T);
    for (int m0 = 0; m0 < n_macro; m0 += band) {
        const int m1 = std::min(n_macro, m0 + band);
        const int i0 = m0 * BAND_MT, i1 = std::min(T, m1 * BAND_MT);
        for (int j0 = i0; j0 < T; j0 += run) {
            const int j1 = std::min(T, j0 + run);
            BandItem it{m0, m1, j0, j1, (int32_t)slot, (int32_t)(slot + (i1 - i0)), 0, 0};
            slot += (i1 - i0) + (j1 - j0);
            int64_t wk = 0;
            for (int I = i0; I < i1; ++I) {
                if (j1 > I) {
                    rows[I].push_back(it.rslot + (I - i0));
                    wk += j1 - std::max(j0, I);
                }
            }
            for (int J = j0; J < j1; ++J)
                if (J > i0)
                    cols[J].push_back(it.cslot + (J - j0));
            all.push_back({it, wk});
        }
    }
    pl.n_records = slot;
    // longest items first, so that the short ones fill in at the end
    std::stable_sort(all.begin(), all.end(),
                     [](const Rec &a, const Rec &b) { return a.work > b.work; });
    items.resize(all.size());
    for (size_t k = 0; k < all.size(); ++k)
        items[k] = all[k].it;
    pl.n_items = (int)items.size();
    rec_start.assign(T + 1, 0);
    rec_idx.clear();
    for (int K = 0; K < T; ++K) {
        rec_start[K] = (int32_t)rec_idx.size();
        rec_idx.insert(rec_idx.end(), rows[K].begin(), rows[K].end());
        rec_idx.insert(rec_idx.end(), cols[K].begin(), cols[K].end());
    }
    rec_start[T] = (int32_t)rec_idx.size();
    return pl;
}

}  // namespace pbk
