// Host driver and C ABI (include/pbsolve.h) of the DSBI Poisson-Boltzmann
// library.  Everything that scales with N runs on the device; the host only
// holds the (m+1) x m Hessenberg matrix of GMRES and its Givens rotations,
// fed by one small device-to-host copy per Arnoldi step.
#include "../../include/pbsolve.h"
#include "pb_ctx.h"
#include "pb_host.h"
#include "pb_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <new>
#include <stdexcept>
#include <system_error>
#include <thread>
#include <vector>

using namespace pbk;

namespace {

int check_params(pb_ctx *c, const pb_params *p, bool solving)
{
    if (!p)
        return fail(c, PB_ERR_ARG, "params is NULL");
    if (!(p->eps_in > 0.0) || !(p->eps_out > 0.0) || !std::isfinite(p->eps_in) ||
        !std::isfinite(p->eps_out))
        return fail(c, PB_ERR_ARG, "eps_in and eps_out must be finite and > 0");
    if (!(p->kappa >= 0.0) || !(p->kappa <= KAPPA_MAX))
        return fail(c, PB_ERR_ARG, "kappa must lie in [0, %g] 1/A", KAPPA_MAX);
    if (solving) {
        if (!(p->tol > 0.0))
            return fail(c, PB_ERR_ARG, "tol must be > 0");
        if (p->restart < 1 || p->restart > MAX_RESTART)
            return fail(c, PB_ERR_ARG, "restart must be in [1, %d]", MAX_RESTART);
        if (p->max_iter < 1)
            return fail(c, PB_ERR_ARG, "max_iter must be >= 1");
        if (p->precision != PB_FP64 && p->precision != PB_FP32_IR)
            return fail(c, PB_ERR_ARG, "precision must be PB_FP64 or PB_FP32_IR");
        if (p->precond_leaf < 0 || p->precond_leaf > PC_MAX_LEAF)
            return fail(c, PB_ERR_ARG, "precond_leaf must be in [0, %d]", PC_MAX_LEAF);
        if (p->precision == PB_FP32_IR) {
            if (p->max_refine < 1)
                return fail(c, PB_ERR_ARG, "max_refine must be >= 1");
            if (!(p->inner_tol > 0.0) || !(p->inner_tol < 1.0))
                return fail(c, PB_ERR_ARG, "inner_tol must be in (0, 1)");
        }
    }
    return PB_OK;
}

// ---- geometry (step 1) with validation --------------------------------------

int setup_geometry(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                   const int32_t *d_tri)
{
    c->pc_leaves = 0;   // a preconditioner and a tree belong to one geometry
    c->t_ready = false;
    if (n_tri <= 0 || n_vert < 3)
        return fail(c, PB_ERR_ARG, "need n_tri > 0 and n_vert >= 3");
    if (n_tri > (int64_t)1 << 30)
        return fail(c, PB_ERR_ARG, "n_tri too large");
    if (!d_vert || !d_tri)
        return fail(c, PB_ERR_ARG, "vertex or triangle array is NULL");
    const int64_t npad = round_up(n_tri, PADN);
    TRY(ensure(c, c->geo, sizeof(double) * NGEO * npad));
    const int nblk = geometry_blocks(npad);
    TRY(ensure(c, c->geo_part, sizeof(double) * GEO_RED * nblk));
    TRY(ensure(c, c->small, sizeof(double) * HSMALL));
    launch_geometry(c->stream, n_vert, n_tri, d_vert, d_tri, as<double>(c->geo), npad, npad,
                    as<double>(c->geo_part), nblk);
    LAUNCHCHK();
    launch_reduce_cols(c->stream, as<double>(c->geo_part), nblk, GEO_RED, as<double>(c->small));
    LAUNCHCHK();
    // coincident centroids (the singular term is dropped by index only)
    const int64_t cap = dup_table_size(n_tri);
    TRY(ensure(c, c->dup_tab, sizeof(int32_t) * (cap + 2)));
    launch_dup_check(c->stream, as<double>(c->geo), n_tri, npad, as<int32_t>(c->dup_tab), cap);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(c->hsmall, c->small.p, sizeof(double) * GEO_RED, hipMemcpyDeviceToHost,
                          c->stream));
    int32_t *hdup = reinterpret_cast<int32_t *>(c->hsmall + HSMALL_DUP);
    HIPCHK(hipMemcpyAsync(hdup, as<int32_t>(c->dup_tab) + cap, sizeof(int32_t) * 2,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const double *r = c->hsmall;
    c->g.g = as<double>(c->geo);
    c->g.n = n_tri;
    c->g.npad = npad;
    if (r[0] != 0.0)
        return fail(c, PB_ERR_GEOMETRY,
                    "%.0f triangle(s) with an out-of-range index, a non-finite vertex or zero area",
                    r[0]);
    if (r[6] != 0.0)
        return fail(c, PB_ERR_GEOMETRY,
                    "%.0f triangle(s) with a centroid coordinate beyond %g A", r[6], COORD_MAX);
    if (hdup[1] != 0)
        return fail(c, PB_ERR_GEOMETRY,
                    "triangle %d shares its centroid with another triangle (%d coincident "
                    "pair(s)): collocation points must be distinct",
                    hdup[0], hdup[1]);
    c->volume = r[1] / 6.0;
    c->area_sum = r[5];
    if (!(c->volume > 0.0))
        return fail(c, PB_ERR_GEOMETRY,
                    "enclosed volume %.6g <= 0: triangles must be counter-clockwise seen from "
                    "outside",
                    c->volume);
    c->center[0] = r[2] / (double)n_tri;
    c->center[1] = r[3] / (double)n_tri;
    c->center[2] = r[4] / (double)n_tri;
    // the mesh's length scale: radius of the sphere of the same area
    c->sigma_min = 1.0 / std::sqrt(c->area_sum / (2.0 * TWO_PI));
    return PB_OK;
}

PairParams pair_params(pb_ctx *c, const pb_params *p)
{
    PairParams pp;
    pp.eps = p->eps_out / p->eps_in;
    pp.kappa = p->kappa;
    pp.cx = c->center[0];
    pp.cy = c->center[1];
    pp.cz = c->center[2];
    pp.sigma = f32_sigma(p->kappa, c->sigma_min);
    return pp;
}

// ---- matvec (steps 3 and 6) -----------------------------------------------------

// Work items of the pairwise sweeps for the current geometry and wave target.
int ensure_sym_plan(pb_ctx *c)
{
    const Geo &g = c->g;
    if (c->sym_plan.npad == g.npad && c->sym_waves == c->f32_waves)
        return PB_OK;
    std::vector<int32_t> items, row_start;
    const SymPlan pl = plan_sym(g.npad, std::max(1, c->f32_waves / (TPB / 64)), items, row_start);
    TRY(ensure(c, c->sym_items, sizeof(int32_t) * items.size()));
    TRY(ensure(c, c->sym_rowstart, sizeof(int32_t) * row_start.size()));
    HIPCHK(hipMemcpyAsync(c->sym_items.p, items.data(), sizeof(int32_t) * items.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->sym_rowstart.p, row_start.data(), sizeof(int32_t) * row_start.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));   // host vectors go out of scope
    c->sym_plan = pl;
    c->sym_waves = c->f32_waves;
    return PB_OK;
}

// Pairwise FP32 sweep: every unordered pair once, both directions.
int apply_pairwise(pb_ctx *c, const pb_params *p, int transpose, const double *x, double *y)
{
    const Geo &g = c->g;
    TRY(ensure_sym_plan(c));
    const SymPlan &pl = c->sym_plan;
    const int64_t T = pl.n_tiles;
    TRY(ensure(c, c->sym_src, sizeof(float) * 12 * g.npad));
    TRY(ensure(c, c->sym_rowpart, sizeof(double) * 2 * TILE * (size_t)pl.n_items));
    TRY(ensure(c, c->sym_colpart,
               sizeof(float) * 2 * TILE * (size_t)std::max<int64_t>(T * (T - 1) / 2, 1)));
    const PairParams pp = pair_params(c, p);
    const double eps = pp.eps, sig = pp.sigma;
    launch_pack_sym(c->stream, g, x, as<float>(c->sym_src), pp.cx, pp.cy, pp.cz, eps, sig,
                    transpose ? 1 : 0);
    LAUNCHCHK();
    {
        ProfScope ps(c, transpose ? PB_KERNEL_PAIRS_FP32_T : PB_KERNEL_PAIRS_FP32,
                     (double)g.n * (double)(g.n - 1));
        launch_pairs_f32_sym(c->stream, as<float>(c->sym_src), as<int32_t>(c->sym_items),
                             pl.n_items, pl.n_tiles, pp, transpose ? 1 : 0,
                             as<double>(c->sym_rowpart), as<float>(c->sym_colpart));
    }
    LAUNCHCHK();
    // lengths in units of 1/sigma: row 1 sums P / (eps sigma^2) forward and
    // -eps P^T / sigma^2 transposed, row 2 sums Q / sigma^3
    const double s1 = transpose ? -sig * sig / eps : eps * sig * sig;
    launch_sym_finish(c->stream, g, as<double>(c->sym_rowpart), as<float>(c->sym_colpart),
                      as<int32_t>(c->sym_rowstart), pl.n_tiles, x, 0.5 * (1.0 + eps),
                      0.5 * (1.0 + 1.0 / eps), transpose ? 1 : 0, s1, sig * sig * sig, y);
    LAUNCHCHK();
    return PB_OK;
}

// Banded pairwise FP32 sweep: work items and record lists for the current
// geometry and item target (target_waves / 64 items).
int ensure_band_plan(pb_ctx *c)
{
    const Geo &g = c->g;
    const int target = std::max(1, c->f32_waves / 64);
    if (c->band_plan.npad == g.npad && c->band_plan.target == target)
        return PB_OK;
    std::vector<BandItem> items;
    std::vector<int32_t> rec_start, rec_idx;
    const BandPlan pl = plan_band(g.npad, target, items, rec_start, rec_idx);
    TRY(ensure(c, c->band_items, sizeof(BandItem) * items.size()));
    TRY(ensure(c, c->band_lists, sizeof(int32_t) * (rec_start.size() + rec_idx.size())));
    HIPCHK(hipMemcpyAsync(c->band_items.p, items.data(), sizeof(BandItem) * items.size(),
                          hipMemcpyHostToDevice, c->stream));
    int32_t *lists = as<int32_t>(c->band_lists);
    HIPCHK(hipMemcpyAsync(lists, rec_start.data(), sizeof(int32_t) * rec_start.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(lists + rec_start.size(), rec_idx.data(),
                          sizeof(int32_t) * rec_idx.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));   // host vectors go out of scope
    c->band_plan = pl;
    return PB_OK;
}

int apply_band(pb_ctx *c, const pb_params *p, int transpose, const double *x, double *y)
{
    const Geo &g = c->g;
    TRY(ensure_band_plan(c));
    const BandPlan &pl = c->band_plan;
    TRY(ensure(c, c->sym_src, sizeof(float) * 12 * g.npad));
    TRY(ensure(c, c->band_recs, sizeof(float) * 2 * TILE * (size_t)std::max<int64_t>(pl.n_records, 1)));
    const PairParams pp = pair_params(c, p);
    const double eps = pp.eps, sig = pp.sigma;
    launch_pack_sym(c->stream, g, x, as<float>(c->sym_src), pp.cx, pp.cy, pp.cz, eps, sig,
                    transpose ? 1 : 0);
    LAUNCHCHK();
    {
        ProfScope ps(c, transpose ? PB_KERNEL_PAIRS_FP32_T : PB_KERNEL_PAIRS_FP32,
                     (double)g.n * (double)(g.n - 1));
        launch_pairs_f32_band(c->stream, as<float>(c->sym_src), as<BandItem>(c->band_items),
                              pl.n_items, pl.n_tiles, pp, transpose ? 1 : 0,
                              as<float>(c->band_recs));
    }
    LAUNCHCHK();
    const int32_t *lists = as<int32_t>(c->band_lists);
    const double s1 = transpose ? -sig * sig / eps : eps * sig * sig;
    launch_band_finish(c->stream, g, as<float>(c->band_recs), lists, lists + pl.n_tiles + 1, x,
                       0.5 * (1.0 + eps), 0.5 * (1.0 + 1.0 / eps), transpose ? 1 : 0, s1,
                       sig * sig * sig, y);
    LAUNCHCHK();
    return PB_OK;
}

// Pairwise FP64 sweep, forward or transposed, on the same work items.
int apply_pairwise64(pb_ctx *c, const pb_params *p, int transpose, const double *x, double *y)
{
    const Geo &g = c->g;
    TRY(ensure_sym_plan(c));
    const SymPlan &pl = c->sym_plan;
    const int64_t T = pl.n_tiles;
    TRY(ensure(c, c->sym_src64, sizeof(double) * 8 * g.npad));
    TRY(ensure(c, c->sym_rowpart, sizeof(double) * 2 * TILE * (size_t)pl.n_items));
    TRY(ensure(c, c->sym_colpart,
               sizeof(double) * 2 * TILE * (size_t)std::max<int64_t>(T * (T - 1) / 2, 1)));
    const PairParams pp = pair_params(c, p);
    const double eps = pp.eps;
    launch_pack_sym64(c->stream, g, x, as<double>(c->sym_src64), transpose ? 1 : 0);
    LAUNCHCHK();
    {
        ProfScope ps(c, transpose ? PB_KERNEL_PAIRS_FP64_T : PB_KERNEL_PAIRS_FP64,
                     (double)g.n * (double)(g.n - 1));
        launch_pairs_f64_sym(c->stream, as<double>(c->sym_src64), as<int32_t>(c->sym_items),
                             pl.n_items, pl.n_tiles, pp, transpose, as<double>(c->sym_rowpart),
                             as<double>(c->sym_colpart));
    }
    LAUNCHCHK();
    launch_sym_finish64(c->stream, g, as<double>(c->sym_rowpart), as<double>(c->sym_colpart),
                        as<int32_t>(c->sym_rowstart), pl.n_tiles, x, 0.5 * (1.0 + eps),
                        0.5 * (1.0 + 1.0 / eps), transpose, y);
    LAUNCHCHK();
    return PB_OK;
}

int apply(pb_ctx *c, const pb_params *p, int precision, int transpose, const double *x, double *y)
{
    const Geo &g = c->g;
    if (c->t_solve && precision == PB_FP64 && !transpose) {   // pb_solve_tree
        TRY(tree_prepare(c, c->t_solve_n0));
        return tree_apply(c, p, c->t_theta, c->t_order, x, y, nullptr);
    }
    if (precision == PB_FP32_IR && c->f32_tpt == PB_SWEEP_PAIRWISE)
        return apply_pairwise(c, p, transpose, x, y);
    if (precision == PB_FP32_IR && c->f32_tpt == PB_SWEEP_BANDED)
        return apply_band(c, p, transpose, x, y);
    if (precision == PB_FP64 && c->f64_kind == PB_SWEEP_PAIRWISE)
        return apply_pairwise64(c, p, transpose, x, y);
    const bool fast32 = precision == PB_FP32_IR && !transpose;
    const Sweep sw = fast32 ? plan_sweep(g.npad, g.npad, c->f32_waves, c->f32_tpt)
                            : plan_sweep(g.npad, g.npad, TARGET_WAVES);
    TRY(ensure(c, c->part, sizeof(double) * 2 * sw.n_chunks * g.npad));
    const PairParams pp = pair_params(c, p);
    const double eps = pp.eps;
    const double npairs = (double)g.n * (double)(g.n - 1);
    double scale1 = 1.0, scale2 = 1.0;
    if (fast32) {
        const double sig = pp.sigma;
        TRY(ensure(c, c->src32, sizeof(float) * 8 * g.npad));
        launch_pack_f32(c->stream, g, x, as<float>(c->src32), 2, pp.cx, pp.cy, pp.cz, eps, sig);
        LAUNCHCHK();
        ProfScope ps(c, PB_KERNEL_PAIRS_FP32, npairs);
        launch_pairs_f32_fwd(c->stream, g, as<float>(c->src32), sw, pp, c->f32_tpt,
                             as<double>(c->part));
        // the reduced form sums row 1 divided by eps, in units of 1/kappa
        scale1 = eps * sig * sig;
        scale2 = sig * sig * sig;
    } else if (precision == PB_FP32_IR) {
        TRY(ensure(c, c->src32, sizeof(float) * 8 * g.npad));
        launch_pack_f32(c->stream, g, x, as<float>(c->src32), 1, pp.cx, pp.cy, pp.cz, eps, 1.0);
        LAUNCHCHK();
        ProfScope ps(c, PB_KERNEL_PAIRS_FP32_T, npairs);
        launch_pairs_f32(c->stream, g, as<float>(c->src32), sw, pp, transpose,
                         as<double>(c->part));
    } else {
        TRY(ensure(c, c->src64, sizeof(double) * 8 * g.npad));
        launch_pack_f64(c->stream, g, x, as<double>(c->src64), transpose ? 1 : 0);
        LAUNCHCHK();
        ProfScope ps(c, transpose ? PB_KERNEL_PAIRS_FP64_T : PB_KERNEL_PAIRS_FP64, npairs);
        launch_pairs_f64(c->stream, g, as<double>(c->src64), sw, pp, transpose,
                         as<double>(c->part));
    }
    LAUNCHCHK();
    launch_matvec_finish(c->stream, g, as<double>(c->part), sw.n_chunks, x, 0.5 * (1.0 + eps),
                         0.5 * (1.0 + 1.0 / eps), transpose, scale1, scale2, y);
    LAUNCHCHK();
    return PB_OK;
}

// ---- block-diagonal leaf preconditioner (Sec. 2.2.4) -------------------------

}  // namespace


namespace {

// Leaves of the current geometry and the inverses of their blocks, in two
// halves: precond_fetch enqueues the copy of the centroids to the host (the
// caller may enqueue more GPU work behind it), precond_finish builds the
// leaves on the host as soon as the copy has landed and inverts the blocks.
int precond_fetch(pb_ctx *c, const pb_params *p)
{
    c->pc_leaves = 0;
    if (p->precond_leaf <= 0)
        return PB_OK;
    const Geo &g = c->g;
    // centroids x, y, z (3 npad doubles, one copy) into pinned staging
    if (c->hgeo_n < (size_t)(3 * g.npad)) {
        if (c->hgeo)
            (void)hipHostFree(c->hgeo);
        c->hgeo = nullptr;
        c->hgeo_n = 0;
        if (hipHostMalloc(reinterpret_cast<void **>(&c->hgeo), sizeof(double) * 3 * g.npad,
                          hipHostMallocDefault) != hipSuccess)
            return fail(c, PB_ERR_OOM, "pinned host staging of %lld doubles",
                        (long long)(3 * g.npad));
        c->hgeo_n = (size_t)(3 * g.npad);
    }
    HIPCHK(hipMemcpyAsync(c->hgeo, g.g, sizeof(double) * 3 * g.npad, hipMemcpyDeviceToHost,
                          c->stream));
    if (!c->ev_fetch)
        HIPCHK(hipEventCreateWithFlags(&c->ev_fetch, hipEventDisableTiming));
    HIPCHK(hipEventRecord(c->ev_fetch, c->stream));
    return PB_OK;
}

int precond_finish(pb_ctx *c, const pb_params *p)
{
    if (p->precond_leaf <= 0)
        return PB_OK;
    const Geo &g = c->g;
    HIPCHK(hipEventSynchronize(c->ev_fetch));
    std::vector<int32_t> perm, start;
    build_leaves(c->hgeo, c->hgeo + g.npad, c->hgeo + 2 * g.npad, g.n, p->precond_leaf, perm,
                 start);
    const int64_t L = (int64_t)start.size() - 1;
    std::vector<int64_t> boff(L + 1, 0);
    for (int64_t l = 0; l < L; ++l) {
        const int64_t m2 = 2 * (int64_t)(start[l + 1] - start[l]);
        boff[l + 1] = boff[l] + m2 * m2;
    }
    const size_t off64 = round_up(sizeof(int32_t) * (g.n + L + 1), 8);
    TRY(ensure(c, c->pc_idx, off64 + sizeof(int64_t) * (L + 1 + 2 * g.n)));
    TRY(ensure(c, c->pc_inv, sizeof(double) * std::max<int64_t>(boff[L], 1)));
    int32_t *dperm = as<int32_t>(c->pc_idx);
    int32_t *dstart = dperm + g.n;
    int64_t *dboff = reinterpret_cast<int64_t *>(static_cast<char *>(c->pc_idx.p) + off64);
    int64_t *dpq = dboff + (L + 1);
    HIPCHK(hipMemcpyAsync(dperm, perm.data(), sizeof(int32_t) * g.n, hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(dstart, start.data(), sizeof(int32_t) * (L + 1), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(dboff, boff.data(), sizeof(int64_t) * (L + 1), hipMemcpyHostToDevice,
                          c->stream));
    launch_pc_index(c->stream, dperm, g.n, dpq);   // phi and psi slots of each element
    LAUNCHCHK();
    launch_pc_build(c->stream, g, dperm, dstart, dboff, L, p->precond_leaf,
                    p->eps_out / p->eps_in, p->kappa, as<double>(c->pc_inv));
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->stream));   // host vectors go out of scope
    c->pc_leaves = L;
    c->pc_perm = dperm;
    c->pc_start = dstart;
    c->pc_boff = dboff;
    c->pc_pidx = dpq;
    c->pc_qidx = dpq + g.n;
    return PB_OK;
}

int setup_precond(pb_ctx *c, const pb_params *p)
{
    TRY(precond_fetch(c, p));
    return precond_finish(c, p);
}

int pc_apply(pb_ctx *c, int transpose, const double *x, double *y)
{
    launch_pc_apply(c->stream, as<double>(c->pc_inv), c->pc_boff, c->pc_pidx, c->pc_qidx,
                    c->pc_start, c->pc_leaves, x, transpose, y);
    LAUNCHCHK();
    return PB_OK;
}

// ---- vectors -------------------------------------------------------------------

struct Vecs {
    int64_t n2 = 0, ld = 0;
    double *x = nullptr, *b = nullptr, *w = nullptr, *r = nullptr, *d = nullptr, *t = nullptr;
    double *lam = nullptr, *aux = nullptr, *pw = nullptr, *pb = nullptr;
    double *V = nullptr;
};

int setup_vectors(pb_ctx *c, int m, Vecs &v)
{
    v.n2 = 2 * c->g.n;
    v.ld = round_up(v.n2, 64);
    TRY(ensure(c, c->vec, sizeof(double) * 10 * v.ld));
    TRY(ensure(c, c->V, sizeof(double) * (m + 1) * v.ld));
    double *base = as<double>(c->vec);
    v.x = base;
    v.b = base + v.ld;
    v.w = base + 2 * v.ld;
    v.r = base + 3 * v.ld;
    v.d = base + 4 * v.ld;
    v.t = base + 5 * v.ld;
    v.lam = base + 6 * v.ld;
    v.aux = base + 7 * v.ld;
    v.pw = base + 8 * v.ld;
    v.pb = base + 9 * v.ld;
    v.V = as<double>(c->V);
    const int nblk = dot_blocks(v.n2);
    TRY(ensure(c, c->dpart, sizeof(double) * (MAX_RESTART + 2) * nblk));
    TRY(ensure(c, c->small, sizeof(double) * HSMALL));
    return PB_OK;
}

// |v|^2 reduced on the device into small[slot]
int norm2_dev(pb_ctx *c, const double *v, int64_t n, int slot)
{
    const int nblk = dot_blocks(n);
    launch_dots(c->stream, nullptr, 0, 0, v, n, as<double>(c->dpart), nblk);
    LAUNCHCHK();
    launch_reduce_cols(c->stream, as<double>(c->dpart), nblk, 1, as<double>(c->small) + slot);
    LAUNCHCHK();
    return PB_OK;
}

int fetch_small(pb_ctx *c, int first, int count)
{
    HIPCHK(hipMemcpyAsync(c->hsmall + first, as<double>(c->small) + first, sizeof(double) * count,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

int norm_host(pb_ctx *c, const double *v, int64_t n, double *out)
{
    const int slot = HSMALL - 1;
    TRY(norm2_dev(c, v, n, slot));
    TRY(fetch_small(c, slot, 1));
    *out = std::sqrt(c->hsmall[slot]);
    return PB_OK;
}

struct GmresStats {
    int iters = 0, mv64 = 0, mv32 = 0;
    double rel = 0.0;
    bool converged = false;
};

// Restarted GMRES(m) (Saad & Schultz) on A x = rhs, A applied in `precision`.
// Arnoldi uses classical Gram-Schmidt with one reorthogonalisation pass
// (CGS2) in FP64 on the device; the Hessenberg least-squares problem is
// solved on the host with Givens rotations.  x holds the start vector unless
// x_zero.  Stops when the true residual |rhs - A x| / |rhs| <= tol.
int gmres(pb_ctx *c, const pb_params *p, int precision, int transpose, const double *rhs,
          double *x, bool x_zero, double tol, int max_iter, Vecs &v, GmresStats &st)
{
    const int m = p->restart;
    const int64_t n2 = v.n2;
    const int nblk = dot_blocks(n2);
    double *small = as<double>(c->small);
    double *h1 = small, *h2 = small + (m + 1), *nb2 = small + 2 * (m + 1);
    double *yv = small + 2 * (m + 1) + 1;
    // Left preconditioning (Sec. 2.2.4): GMRES on M^-1 A x = M^-1 rhs.
    const bool pc = c->pc_leaves > 0;
    const double *prhs = rhs;
    if (pc) {
        TRY(pc_apply(c, transpose, rhs, v.pb));
        prhs = v.pb;
    }
    double *rr = pc ? v.pw : v.r;   // (preconditioned) residual
    double *ww = pc ? v.pw : v.w;   // (preconditioned) new Krylov direction
    double bnorm;
    TRY(norm_host(c, prhs, n2, &bnorm));
    st = GmresStats();
    if (!std::isfinite(bnorm))
        return fail(c, PB_ERR_GEOMETRY, "non-finite right-hand side");
    if (bnorm == 0.0) {
        launch_fill(c->stream, x, 0.0, n2);
        LAUNCHCHK();
        st.converged = true;
        return PB_OK;
    }
    std::vector<double> H((m + 1) * m), cs(m), sn(m), gv(m + 1), yh(m);
    bool zero_start = x_zero;
    double prev_rel = 0.0;
    if (x_zero) {
        launch_fill(c->stream, x, 0.0, n2);
        LAUNCHCHK();
    }
    for (;;) {
        // r0 = rhs - A x  (r0 = rhs when starting from zero)
        double beta;
        if (zero_start) {
            HIPCHK(hipMemcpyAsync(rr, prhs, sizeof(double) * n2, hipMemcpyDeviceToDevice,
                                  c->stream));
            beta = bnorm;
        } else {
            TRY(apply(c, p, precision, transpose, x, v.w));
            if (precision == PB_FP64) st.mv64++; else st.mv32++;
            launch_sub(c->stream, rhs, v.w, v.r, n2);
            LAUNCHCHK();
            if (pc)
                TRY(pc_apply(c, transpose, v.r, rr));
            TRY(norm_host(c, rr, n2, &beta));
        }
        zero_start = false;
        if (!std::isfinite(beta))
            return fail(c, PB_ERR_GEOMETRY,
                        "non-finite residual (coincident collocation points or a charge on "
                        "the surface?)");
        st.rel = beta / bnorm;
        if (st.rel <= tol) {
            st.converged = true;
            return PB_OK;
        }
        if (st.iters >= max_iter)
            return PB_OK;
        // An FP32 operator resolves the residual only to about 1e-6..1e-7 of
        // |rhs|: a restart cycle that no longer gains 10 % ends the inner
        // solve and leaves the rest to the FP64 refinement around it.
        if (precision == PB_FP32_IR && prev_rel > 0.0 && st.rel > 0.9 * prev_rel)
            return PB_OK;
        prev_rel = st.rel;
        // V_0 = r0 / beta
        TRY(norm2_dev(c, rr, n2, 2 * (m + 1)));
        launch_scale_inv_sqrt(c->stream, rr, nb2, v.V, n2);
        LAUNCHCHK();
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = v.V + (int64_t)j * v.ld;
            TRY(apply(c, p, precision, transpose, vj, v.w));
            st.iters++;
            if (precision == PB_FP64) st.mv64++; else st.mv32++;
            if (pc)
                TRY(pc_apply(c, transpose, v.w, ww));
            // CGS pass 1 and 2
            launch_dots(c->stream, v.V, v.ld, j + 1, ww, n2, as<double>(c->dpart), nblk);
            LAUNCHCHK();
            launch_reduce_cols(c->stream, as<double>(c->dpart), nblk, j + 1, h1);
            LAUNCHCHK();
            launch_sub_basis(c->stream, v.V, v.ld, j + 1, h1, ww, n2);
            LAUNCHCHK();
            launch_dots(c->stream, v.V, v.ld, j + 1, ww, n2, as<double>(c->dpart), nblk);
            LAUNCHCHK();
            launch_reduce_cols(c->stream, as<double>(c->dpart), nblk, j + 1, h2);
            LAUNCHCHK();
            launch_sub_basis(c->stream, v.V, v.ld, j + 1, h2, ww, n2);
            LAUNCHCHK();
            TRY(norm2_dev(c, ww, n2, 2 * (m + 1)));
            launch_scale_inv_sqrt(c->stream, ww, nb2, v.V + (int64_t)(j + 1) * v.ld, n2);
            LAUNCHCHK();
            TRY(fetch_small(c, 0, 2 * (m + 1) + 1));
            const double *hh = c->hsmall;
            for (int i = 0; i <= j; ++i)
                H[i * m + j] = hh[i] + hh[(m + 1) + i];
            const double hn = std::sqrt(hh[2 * (m + 1)]);
            if (!std::isfinite(hn))
                return fail(c, PB_ERR_GEOMETRY,
                            "non-finite Arnoldi vector (coincident collocation points?)");
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t;
            }
            const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
            cs[j] = H[j * m + j] / den;
            sn[j] = H[(j + 1) * m + j] / den;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            if (std::fabs(gv[j + 1]) / bnorm <= tol || st.iters >= max_iter || hn == 0.0)
                break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int l = i + 1; l < k; ++l)
                s -= H[i * m + l] * yh[l];
            yh[i] = s / H[i * m + i];
        }
        std::memcpy(c->hsmall + (yv - small), yh.data(), sizeof(double) * k);
        HIPCHK(hipMemcpyAsync(yv, c->hsmall + (yv - small), sizeof(double) * k,
                              hipMemcpyHostToDevice, c->stream));
        launch_add_basis(c->stream, v.V, v.ld, k, yv, x, n2);
        LAUNCHCHK();
        // the host staging row is reused by the next fetch: drain first
        HIPCHK(hipStreamSynchronize(c->stream));
        // Inside iterative refinement the FP64 residual of the updated
        // iterate is taken next by the caller, which is the stronger test:
        // a converged Arnoldi estimate ends the FP32 solve without an FP32
        // confirmation matvec.
        if (precision == PB_FP32_IR && k > 0 && std::fabs(gv[k]) / bnorm <= tol) {
            st.rel = std::fabs(gv[k]) / bnorm;
            st.converged = true;
            return PB_OK;
        }
    }
}

// ---- charges: inside check, sources (step 2), energy (step 5) -----------------

// Discrete solid angle of the surface at every charge (one N x Nc sweep with
// unit potential and zero flux); the result is copied to pinned staging and
// judged by charges_inside_verdict after the stream drains.
int launch_charges_inside(pb_ctx *c, const pb_params *p, int64_t nc, const double *d_pos,
                         Vecs &v)
{
    const Geo &g = c->g;
    const Sweep sw = plan_sweep(nc, g.npad, TARGET_WAVES);
    const int64_t ncpad = (int64_t)sw.n_tblocks * TPB;
    TRY(ensure(c, c->chg_part, sizeof(double) * sw.n_chunks * ncpad));
    TRY(ensure(c, c->chg_per, sizeof(double) * ncpad));
    TRY(ensure(c, c->src64, sizeof(double) * 8 * g.npad));
    // unit potential, zero flux: the stream carries m_j = a_j n_j
    launch_fill(c->stream, v.t, 1.0, g.n);
    LAUNCHCHK();
    launch_fill(c->stream, v.t + g.n, 0.0, g.n);
    LAUNCHCHK();
    launch_pack_f64(c->stream, g, v.t, as<double>(c->src64), 0);
    LAUNCHCHK();
    {
        ProfScope ps(c, PB_KERNEL_CHARGE, (double)g.n * (double)nc);
        launch_charge_pairs(c->stream, g, as<double>(c->src64), nc, d_pos, sw, pair_params(c, p),
                            1, as<double>(c->chg_part), ncpad);
    }
    LAUNCHCHK();
    launch_charge_finish(c->stream, as<double>(c->chg_part), sw.n_chunks, nc, ncpad, nullptr,
                         1.0, as<double>(c->chg_per), nullptr);
    LAUNCHCHK();
    if (c->hchg_n < (size_t)nc) {
        if (c->hchg)
            (void)hipHostFree(c->hchg);
        c->hchg = nullptr;
        c->hchg_n = 0;
        if (hipHostMalloc(reinterpret_cast<void **>(&c->hchg), sizeof(double) * nc,
                          hipHostMallocDefault) != hipSuccess)
            return fail(c, PB_ERR_OOM, "pinned host staging of %lld doubles", (long long)nc);
        c->hchg_n = (size_t)nc;
    }
    HIPCHK(hipMemcpyAsync(c->hchg, c->chg_per.p, sizeof(double) * nc, hipMemcpyDeviceToHost,
                          c->stream));
    return PB_OK;
}

// The verdict of launch_charges_inside, once the stream has drained.
int charges_inside_verdict(pb_ctx *c, int64_t nc)
{
    const double *omega = c->hchg;
    for (int64_t k = 0; k < nc; ++k) {
        // discrete solid angle: ~4 pi inside, ~0 outside
        if (!(omega[k] >= TWO_PI))
            return fail(c, PB_ERR_CHARGE,
                        "charge %lld is not inside the surface (solid angle %.4g, need >= 2 pi)",
                        (long long)k, omega[k]);
    }
    return PB_OK;
}

int energy_dev(pb_ctx *c, const pb_params *p, int64_t nc, const double *d_pos, const double *d_q,
               const double *x, double *e_out)
{
    const Geo &g = c->g;
    const Sweep sw = plan_sweep(nc, g.npad, TARGET_WAVES);
    const int64_t ncpad = (int64_t)sw.n_tblocks * TPB;
    TRY(ensure(c, c->chg_part, sizeof(double) * sw.n_chunks * ncpad));
    TRY(ensure(c, c->src64, sizeof(double) * 8 * g.npad));
    TRY(ensure(c, c->small, sizeof(double) * HSMALL));
    launch_pack_f64(c->stream, g, x, as<double>(c->src64), 0);
    LAUNCHCHK();
    {
        ProfScope ps(c, PB_KERNEL_CHARGE, (double)g.n * (double)nc);
        launch_charge_pairs(c->stream, g, as<double>(c->src64), nc, d_pos, sw, pair_params(c, p),
                            0, as<double>(c->chg_part), ncpad);
    }
    LAUNCHCHK();
    const int slot = HSMALL - 2;
    TRY(ensure(c, c->chg_per, sizeof(double) * ncpad));
    // E = (1/2) sum_k q_k phi_reac(y_k) in kcal/mol; the pair sums carry 4 pi K
    launch_charge_finish(c->stream, as<double>(c->chg_part), sw.n_chunks, nc, ncpad, d_q,
                         0.5 * C_UNITS, as<double>(c->chg_per), as<double>(c->small) + slot);
    LAUNCHCHK();
    TRY(fetch_small(c, slot, 1));
    *e_out = c->hsmall[slot];
    return PB_OK;
}

int check_charges_args(pb_ctx *c, int64_t nc, const void *pos, const void *q)
{
    if (nc <= 0)
        return fail(c, PB_ERR_ARG, "need at least one charge");
    if (!pos || !q)
        return fail(c, PB_ERR_ARG, "charge position or value array is NULL");
    return PB_OK;
}

struct SolveStats {
    int iters = 0, mv64 = 0, mv32 = 0, refinements = 0, status = PB_OK;
    double rel = 0.0;
};

// A x = rhs (A^T x = rhs when transposed) to p->tol: FP64 GMRES, or FP32
// inner GMRES solves inside FP64 iterative refinement (r = rhs - A x in
// FP64; inner solve A d = r in FP32 pair arithmetic to inner_tol; x += d).
// Uses v.w, v.r, v.t, v.d and the Krylov basis; rhs and x must be other slots.
int solve_system(pb_ctx *c, const pb_params *p, int transpose, const double *rhs, double *x,
                 Vecs &v, SolveStats &out)
{
    out = SolveStats();
    GmresStats st;
    if (p->precision == PB_FP64) {
        TRY(gmres(c, p, PB_FP64, transpose, rhs, x, true, p->tol, p->max_iter, v, st));
        out.iters = st.iters;
        out.mv64 = st.mv64;
        out.rel = st.rel;
        out.status = st.converged ? PB_OK : PB_NOT_CONVERGED;
        return PB_OK;
    }
    // With the preconditioner on, the outer test uses the same left-
    // preconditioned norm |M^-1 (rhs - A x)| / |M^-1 rhs| as the inner solves.
    const bool pc = c->pc_leaves > 0;
    double bnorm;
    if (pc) {
        TRY(pc_apply(c, transpose, rhs, v.pw));
        TRY(norm_host(c, v.pw, v.n2, &bnorm));
    } else {
        TRY(norm_host(c, rhs, v.n2, &bnorm));
    }
    launch_fill(c->stream, x, 0.0, v.n2);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(v.r, rhs, sizeof(double) * v.n2, hipMemcpyDeviceToDevice, c->stream));
    double rnorm = bnorm;
    out.status = PB_NOT_CONVERGED;
    for (;;) {
        out.rel = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        if (out.rel <= p->tol) {
            out.status = PB_OK;
            break;
        }
        if (out.refinements >= p->max_refine || out.iters >= p->max_iter)
            break;
        HIPCHK(hipMemcpyAsync(v.t, v.r, sizeof(double) * v.n2, hipMemcpyDeviceToDevice,
                              c->stream));
        // a correction solve only has to close the gap between |r| and tol |b|
        double eta = std::max(p->inner_tol, 1e-7);
        if (out.refinements > 0 && rnorm > 0.0)
            eta = std::max(eta, std::min(0.5, 0.3 * p->tol * bnorm / rnorm));
        TRY(gmres(c, p, PB_FP32_IR, transpose, v.t, v.d, true, eta, p->max_iter - out.iters, v,
                  st));
        out.iters += st.iters;
        out.mv32 += st.mv32;
        launch_add(c->stream, x, v.d, v.n2);
        LAUNCHCHK();
        out.refinements++;
        TRY(apply(c, p, PB_FP64, transpose, x, v.w));
        out.mv64++;
        launch_sub(c->stream, rhs, v.w, v.r, v.n2);
        LAUNCHCHK();
        if (pc) {
            TRY(pc_apply(c, transpose, v.r, v.pw));
            TRY(norm_host(c, v.pw, v.n2, &rnorm));
        } else {
            TRY(norm_host(c, v.r, v.n2, &rnorm));
        }
        if (!std::isfinite(rnorm))
            return fail(c, PB_ERR_GEOMETRY, "non-finite residual in refinement");
    }
    return PB_OK;
}

// Steps 1, 2 and the forward solve on device-resident inputs; leaves the
// solution in v.x.
int forward_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                const int32_t *d_tri, int64_t nc, const double *d_pos, const double *d_q,
                const pb_params *p, Vecs &v, SolveStats &ss)
{
    TRY(check_params(c, p, true));
    TRY(check_charges_args(c, nc, d_pos, d_q));
    TRY(setup_geometry(c, n_vert, n_tri, d_vert, d_tri));
    TRY(setup_vectors(c, p->restart, v));
    // The centroid copy goes first; the charge check and the sources run on
    // the device while the host builds the preconditioner's leaves.
    TRY(precond_fetch(c, p));
    TRY(launch_charges_inside(c, p, nc, d_pos, v));
    {
        ProfScope ps(c, PB_KERNEL_SOURCE, (double)c->g.n * (double)nc);
        launch_source(c->stream, c->g, nc, d_pos, d_q, p->eps_in, v.b);
    }
    LAUNCHCHK();
    TRY(precond_finish(c, p));
    HIPCHK(hipStreamSynchronize(c->stream));
    TRY(charges_inside_verdict(c, nc));
    TRY(solve_system(c, p, 0, v.b, v.x, v, ss));
    return PB_OK;
}

void fill_info(pb_info *info, double e, const SolveStats &f, const SolveStats *a)
{
    if (!info)
        return;
    info->e_solv = e;
    info->rel_residual = f.rel;
    info->iters = f.iters;
    info->matvecs_fp64 = f.mv64 + (a ? a->mv64 : 0);
    info->matvecs_fp32 = f.mv32 + (a ? a->mv32 : 0);
    info->refinements = f.refinements;
    info->adjoint_iters = a ? a->iters : 0;
    int st = f.status;
    if (a && a->status != PB_OK)
        st = a->status;
    info->status = st;
}

// Whole path on device-resident inputs.
int solve_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
              const int32_t *d_tri, int64_t nc, const double *d_pos, const double *d_q,
              const pb_params *p, double *d_phi, double *d_dphi, pb_info *info)
{
    Vecs v;
    SolveStats ss;
    TRY(forward_dev(c, n_vert, n_tri, d_vert, d_tri, nc, d_pos, d_q, p, v, ss));
    double e = 0.0;
    TRY(energy_dev(c, p, nc, d_pos, d_q, v.x, &e));
    if (d_phi)
        HIPCHK(hipMemcpyAsync(d_phi, v.x, sizeof(double) * n_tri, hipMemcpyDeviceToDevice,
                              c->stream));
    if (d_dphi)
        HIPCHK(hipMemcpyAsync(d_dphi, v.x + n_tri, sizeof(double) * n_tri,
                              hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    fill_info(info, e, ss, nullptr);
    if (ss.status == PB_NOT_CONVERGED)
        fail(c, PB_NOT_CONVERGED, "GMRES stopped at relative residual %.3e > tol %.3e", ss.rel,
             p->tol);
    return ss.status;
}

// Forward solve, adjoint solve A^T lam' = B'^T q and the gradient sweep.
int forces_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
               const int32_t *d_tri, int64_t nc, const double *d_pos, const double *d_q,
               const pb_params *p, double *d_dpos, double *d_dq, pb_info *info)
{
    if (!d_dpos || !d_dq)
        return fail(c, PB_ERR_ARG, "gradient outputs are NULL");
    Vecs v;
    SolveStats fs, as_;
    TRY(forward_dev(c, n_vert, n_tri, d_vert, d_tri, nc, d_pos, d_q, p, v, fs));
    const Geo &g = c->g;
    const PairParams pp = pair_params(c, p);
    {
        ProfScope ps(c, PB_KERNEL_CHARGE, (double)g.n * (double)nc);
        launch_adjoint_rhs(c->stream, g, nc, d_pos, d_q, pp.eps, pp.kappa, v.aux);
    }
    LAUNCHCHK();
    TRY(solve_system(c, p, 1, v.aux, v.lam, v, as_));
    const Sweep sw = plan_sweep(nc, g.npad, TARGET_WAVES);
    const int64_t ncpad = (int64_t)sw.n_tblocks * TPB;
    TRY(ensure(c, c->chg_part, sizeof(double) * 8 * sw.n_chunks * ncpad));
    TRY(ensure(c, c->src64, sizeof(double) * 16 * g.npad));
    double *fwd = as<double>(c->src64), *adj = fwd + 8 * g.npad;
    launch_pack_f64(c->stream, g, v.x, fwd, 0);
    LAUNCHCHK();
    launch_pack_f64(c->stream, g, v.lam, adj, 1);
    LAUNCHCHK();
    {
        ProfScope ps(c, PB_KERNEL_CHARGE, (double)g.n * (double)nc);
        launch_force_pairs(c->stream, fwd, adj, nc, d_pos, sw, pp, as<double>(c->chg_part), ncpad);
    }
    LAUNCHCHK();
    const int slot = HSMALL - 3;
    TRY(ensure(c, c->chg_per, sizeof(double) * ncpad));
    launch_force_finish(c->stream, as<double>(c->chg_part), sw.n_chunks, nc, ncpad, d_q,
                        0.5 * C_UNITS, 1.0 / (4.0 * M_PI * p->eps_in), d_dpos, d_dq,
                        as<double>(c->chg_per), as<double>(c->small) + slot);
    LAUNCHCHK();
    TRY(fetch_small(c, slot, 1));
    fill_info(info, c->hsmall[slot], fs, &as_);
    if (info && info->status == PB_NOT_CONVERGED)
        fail(c, PB_NOT_CONVERGED, "forward or adjoint GMRES did not reach tol %.3e", p->tol);
    return info ? info->status : (fs.status != PB_OK ? fs.status : as_.status);
}

// Host inputs -> context buffers.
int upload_surface(pb_ctx *c, const pb_surface *s, const double **dv, const int32_t **dt)
{
    if (!s || !s->vert || !s->tri)
        return fail(c, PB_ERR_ARG, "surface or its arrays are NULL");
    if (s->n_tri <= 0 || s->n_vert < 3)
        return fail(c, PB_ERR_ARG, "need n_tri > 0 and n_vert >= 3");
    TRY(ensure(c, c->in_vert, sizeof(double) * 3 * s->n_vert));
    TRY(ensure(c, c->in_tri, sizeof(int32_t) * 3 * s->n_tri));
    HIPCHK(hipMemcpyAsync(c->in_vert.p, s->vert, sizeof(double) * 3 * s->n_vert,
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->in_tri.p, s->tri, sizeof(int32_t) * 3 * s->n_tri,
                          hipMemcpyHostToDevice, c->stream));
    *dv = as<double>(c->in_vert);
    *dt = as<int32_t>(c->in_tri);
    return PB_OK;
}

int upload_charges(pb_ctx *c, const pb_charges *q, const double **dp, const double **dq)
{
    if (!q)
        return fail(c, PB_ERR_ARG, "charges is NULL");
    TRY(check_charges_args(c, q->n, q->pos, q->q));
    TRY(ensure(c, c->in_pos, sizeof(double) * 3 * q->n));
    TRY(ensure(c, c->in_q, sizeof(double) * q->n));
    HIPCHK(hipMemcpyAsync(c->in_pos.p, q->pos, sizeof(double) * 3 * q->n, hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(c->in_q.p, q->q, sizeof(double) * q->n, hipMemcpyHostToDevice,
                          c->stream));
    *dp = as<double>(c->in_pos);
    *dq = as<double>(c->in_q);
    return PB_OK;
}

int enter(pb_ctx *c)
{
    if (!c)
        return PB_ERR_ARG;
    HIPCHK(hipSetDevice(c->device));
    return PB_OK;
}

// Every entry point returns through here: drain the stream and fold the
// recorded kernel timings in, whatever the status.
// Runs an entry point's body; no exception crosses the C ABI (host
// allocations, thread creation): they become status codes.
template <typename F>
int guarded(pb_ctx *c, F &&body)
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return c ? fail(c, PB_ERR_OOM, "host memory exhausted") : PB_ERR_OOM;
    } catch (const std::exception &e) {
        return c ? fail(c, PB_ERR_HIP, "host error: %s", e.what()) : PB_ERR_HIP;
    } catch (...) {
        return c ? fail(c, PB_ERR_HIP, "host error") : PB_ERR_HIP;
    }
}

int leave(pb_ctx *c, int st)
{
    if (c && !c->marks.empty()) {
        if (hipStreamSynchronize(c->stream) == hipSuccess)
            prof_collect(c);
        else
            c->marks.clear();
    }
    return st;
}

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ======================= C ABI ===================================================

extern "C" {

int pb_abi_version(void) { return PB_ABI_VERSION; }

int pb_create(int device, void *hip_stream, pb_ctx **out)
{
    if (!out)
        return PB_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return PB_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess)
        return PB_ERR_HIP;
    pb_ctx *c = new (std::nothrow) pb_ctx();
    if (!c)
        return PB_ERR_OOM;
    c->device = device;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return PB_ERR_HIP;
        }
        c->own_stream = true;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->hsmall), sizeof(double) * HSMALL,
                      hipHostMallocDefault) != hipSuccess) {
        if (c->own_stream)
            (void)hipStreamDestroy(c->stream);
        delete c;
        return PB_ERR_OOM;
    }
    // the device address of this GPU's no-allocation scratch, once per device
    const int na = noalloc_init(device);
    if (na != PB_OK) {
        (void)hipHostFree(c->hsmall);
        if (c->own_stream)
            (void)hipStreamDestroy(c->stream);
        delete c;
        return na;
    }
    *out = c;
    return PB_OK;
}

void pb_destroy(pb_ctx *c)
{
    if (!c)
        return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf *bufs[] = {&c->geo, &c->geo_part, &c->src64, &c->src32, &c->part, &c->vec,
                      &c->V, &c->small, &c->dpart, &c->chg_part, &c->chg_per, &c->in_vert,
                      &c->in_tri, &c->in_pos, &c->in_q, &c->io_x, &c->io_y, &c->pc_idx,
                      &c->pc_inv, &c->b_geo, &c->b_desc, &c->b_map, &c->b_items, &c->b_src,
                      &c->b_part, &c->b_vec, &c->b_V, &c->b_state, &c->b_red, &c->b_chg,
                      &c->b_pc_idx, &c->b_pc_inv, &c->sym_src, &c->sym_items,
                      &c->sym_rowstart, &c->sym_rowpart, &c->sym_colpart, &c->sym_src64,
                      &c->t_nodes,
                      &c->t_ctr, &c->t_perm, &c->t_geo, &c->t_wv, &c->t_out, &c->t_mom,
                      &c->t_cnt, &c->b_sitems, &c->b_rs, &c->b_srow, &c->b_scol,
                      &c->b_pc_sys, &c->dup_tab, &c->band_items, &c->band_lists,
                      &c->band_recs, &c->probe_out};
    for (DevBuf *b : bufs)
        if (b->p)
            (void)hipFree(b->p);
    if (c->hsmall)
        (void)hipHostFree(c->hsmall);
    if (c->hgeo)
        (void)hipHostFree(c->hgeo);
    if (c->hchg)
        (void)hipHostFree(c->hchg);
    if (c->ev_fetch)
        (void)hipEventDestroy(c->ev_fetch);
    for (hipEvent_t e : c->ev_pool)
        (void)hipEventDestroy(e);
    if (c->own_stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *pb_last_error(const pb_ctx *c)
{
    if (!c)
        return "NULL context";
    return c->err.msg.c_str();
}

static int pb_geometry_impl(pb_ctx *c, const pb_surface *s, double *cen, double *nrm, double *area)
{
    TRY(enter(c));
    if (!cen || !nrm || !area)
        return fail(c, PB_ERR_ARG, "output arrays are NULL");
    const double *dv;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    const int64_t n = c->g.n, np = c->g.npad;
    std::vector<double> h(NGEO * np);
    HIPCHK(hipMemcpyAsync(h.data(), c->g.g, sizeof(double) * NGEO * np, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 3; ++k) {
            cen[3 * i + k] = h[k * np + i];
            nrm[3 * i + k] = h[(3 + k) * np + i];
        }
        area[i] = h[6 * np + i];
    }
    return PB_OK;
}

static int pb_source_impl(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p, double *b)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!b)
        return fail(c, PB_ERR_ARG, "output b is NULL");
    const double *dv, *dp, *dq;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(upload_charges(c, q, &dp, &dq));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    TRY(ensure(c, c->io_y, sizeof(double) * 2 * s->n_tri));
    launch_source(c->stream, c->g, q->n, dp, dq, p->eps_in, as<double>(c->io_y));
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(b, c->io_y.p, sizeof(double) * 2 * s->n_tri, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

static int pb_matvec_impl(pb_ctx *c, const pb_surface *s, const pb_params *p, const double *x, double *y,
              int transpose, int precision)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!x || !y)
        return fail(c, PB_ERR_ARG, "x or y is NULL");
    if (precision != PB_FP64 && precision != PB_FP32_IR)
        return fail(c, PB_ERR_ARG, "precision must be PB_FP64 or PB_FP32_IR");
    const double *dv;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    const int64_t n2 = 2 * s->n_tri;
    TRY(ensure(c, c->io_x, sizeof(double) * n2));
    TRY(ensure(c, c->io_y, sizeof(double) * n2));
    HIPCHK(hipMemcpyAsync(c->io_x.p, x, sizeof(double) * n2, hipMemcpyHostToDevice, c->stream));
    TRY(apply(c, p, precision, transpose ? 1 : 0, as<double>(c->io_x), as<double>(c->io_y)));
    HIPCHK(hipMemcpyAsync(y, c->io_y.p, sizeof(double) * n2, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

static int pb_matvec_tree_impl(pb_ctx *c, const pb_surface *s, const pb_params *p, double theta,
                               int order, int leaf_size, const double *x, double *y,
                               int64_t *counts)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!x || !y)
        return fail(c, PB_ERR_ARG, "x or y is NULL");
    if (!(theta >= 0.0 && theta < 1.0))
        return fail(c, PB_ERR_ARG, "theta must lie in [0, 1)");
    if (order < 0 || order > 5)
        return fail(c, PB_ERR_ARG, "treecode order must be 0..5");
    if (leaf_size < 1)
        return fail(c, PB_ERR_ARG, "leaf_size must be >= 1");
    const double *dv;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    const int64_t n2 = 2 * s->n_tri;
    TRY(ensure(c, c->io_x, sizeof(double) * n2));
    TRY(ensure(c, c->io_y, sizeof(double) * n2));
    HIPCHK(hipMemcpyAsync(c->io_x.p, x, sizeof(double) * n2, hipMemcpyHostToDevice, c->stream));
    TRY(tree_matvec(c, p, theta, order, leaf_size, as<double>(c->io_x), as<double>(c->io_y),
                    counts));
    HIPCHK(hipMemcpyAsync(y, c->io_y.p, sizeof(double) * n2, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

static int pb_matvec_dev_impl(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, const pb_params *p, const double *d_x, double *d_y,
                  int transpose, int precision)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!d_x || !d_y)
        return fail(c, PB_ERR_ARG, "x or y is NULL");
    if (precision != PB_FP64 && precision != PB_FP32_IR)
        return fail(c, PB_ERR_ARG, "precision must be PB_FP64 or PB_FP32_IR");
    TRY(setup_geometry(c, n_vert, n_tri, d_vert, d_tri));
    TRY(apply(c, p, precision, transpose ? 1 : 0, d_x, d_y));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

static int pb_source_dev_impl(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                              const int32_t *d_tri, int64_t nc, const double *d_pos,
                              const double *d_q, const pb_params *p, double *d_b)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    TRY(check_charges_args(c, nc, d_pos, d_q));
    if (!d_b)
        return fail(c, PB_ERR_ARG, "output b is NULL");
    TRY(setup_geometry(c, n_vert, n_tri, d_vert, d_tri));
    launch_source(c->stream, c->g, nc, d_pos, d_q, p->eps_in, d_b);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

static int pb_energy_dev_impl(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                              const int32_t *d_tri, int64_t nc, const double *d_pos,
                              const double *d_q, const pb_params *p, const double *d_phi,
                              const double *d_dphi, double *e_solv)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    TRY(check_charges_args(c, nc, d_pos, d_q));
    if (!d_phi || !d_dphi || !e_solv)
        return fail(c, PB_ERR_ARG, "phi, dphi or e_solv is NULL");
    TRY(setup_geometry(c, n_vert, n_tri, d_vert, d_tri));
    TRY(ensure(c, c->io_x, sizeof(double) * 2 * n_tri));
    HIPCHK(hipMemcpyAsync(c->io_x.p, d_phi, sizeof(double) * n_tri, hipMemcpyDeviceToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(as<double>(c->io_x) + n_tri, d_dphi, sizeof(double) * n_tri,
                          hipMemcpyDeviceToDevice, c->stream));
    return energy_dev(c, p, nc, d_pos, d_q, as<double>(c->io_x), e_solv);
}

static int pb_energy_impl(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
              const double *phi, const double *dphi, double *e_solv)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!phi || !dphi || !e_solv)
        return fail(c, PB_ERR_ARG, "phi, dphi or e_solv is NULL");
    const double *dv, *dp, *dq;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(upload_charges(c, q, &dp, &dq));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    const int64_t n = s->n_tri;
    TRY(ensure(c, c->io_x, sizeof(double) * 2 * n));
    HIPCHK(hipMemcpyAsync(c->io_x.p, phi, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(as<double>(c->io_x) + n, dphi, sizeof(double) * n,
                          hipMemcpyHostToDevice, c->stream));
    return energy_dev(c, p, q->n, dp, dq, as<double>(c->io_x), e_solv);
}

static int pb_solve_impl(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
             double *phi, double *dphi, pb_info *info)
{
    const double t0 = now_s();
    TRY(enter(c));
    const double *dv, *dp, *dq;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(upload_charges(c, q, &dp, &dq));
    const int64_t n = s->n_tri;
    double *dphi_d = nullptr;
    if (phi || dphi) {
        TRY(ensure(c, c->io_y, sizeof(double) * 2 * n));
        dphi_d = as<double>(c->io_y);
    }
    const int st = solve_dev(c, s->n_vert, s->n_tri, dv, dt, q->n, dp, dq, p, dphi_d,
                             dphi_d ? dphi_d + n : nullptr, info);
    if (st < 0)
        return st;
    if (phi)
        HIPCHK(hipMemcpyAsync(phi, dphi_d, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    if (dphi)
        HIPCHK(hipMemcpyAsync(dphi, dphi_d + n, sizeof(double) * n, hipMemcpyDeviceToHost,
                              c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (info)
        info->seconds = now_s() - t0;
    return st;
}

static int pb_solve_tree_impl(pb_ctx *c, const pb_surface *s, const pb_charges *q,
                              const pb_params *p, double theta, int order, int leaf_size,
                              double *phi, double *dphi, pb_info *info)
{
    if (!c)
        return PB_ERR_ARG;
    if (!(theta >= 0.0 && theta < 1.0))
        return fail(c, PB_ERR_ARG, "theta must lie in [0, 1)");
    if (order < 0 || order > 5)
        return fail(c, PB_ERR_ARG, "treecode order must be 0..5");
    if (leaf_size < 1)
        return fail(c, PB_ERR_ARG, "leaf_size must be >= 1");
    if (p && p->precision != PB_FP64)
        return fail(c, PB_ERR_ARG, "treecode solves run in FP64 (precision PB_FP64)");
    struct Off {
        pb_ctx *c;
        ~Off() { c->t_solve = false; }
    } off{c};
    c->t_solve = true;
    c->t_theta = theta;
    c->t_order = order;
    c->t_solve_n0 = leaf_size;
    return pb_solve_impl(c, s, q, p, phi, dphi, info);
}

static int pb_forces_impl(pb_ctx *c, const pb_surface *s, const pb_charges *q,
                          const pb_params *p, double *dE_dpos, double *dE_dq, pb_info *info)
{
    const double t0 = now_s();
    TRY(enter(c));
    if (!dE_dpos || !dE_dq)
        return fail(c, PB_ERR_ARG, "gradient outputs are NULL");
    const double *dv, *dp, *dq;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(upload_charges(c, q, &dp, &dq));
    TRY(ensure(c, c->io_y, sizeof(double) * 4 * q->n));
    double *gpos = as<double>(c->io_y), *gq = gpos + 3 * q->n;
    const int st = forces_dev(c, s->n_vert, s->n_tri, dv, dt, q->n, dp, dq, p, gpos, gq, info);
    if (st < 0)
        return st;
    HIPCHK(hipMemcpyAsync(dE_dpos, gpos, sizeof(double) * 3 * q->n, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(dE_dq, gq, sizeof(double) * q->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (info)
        info->seconds = now_s() - t0;
    return st;
}

static int pb_forces_dev_impl(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                              const int32_t *d_tri, int64_t n_charges, const double *d_pos,
                              const double *d_q, const pb_params *p, double *d_dE_dpos,
                              double *d_dE_dq, pb_info *info)
{
    const double t0 = now_s();
    TRY(enter(c));
    const int st = forces_dev(c, n_vert, n_tri, d_vert, d_tri, n_charges, d_pos, d_q, p,
                              d_dE_dpos, d_dE_dq, info);
    if (info && st >= 0)
        info->seconds = now_s() - t0;
    return st;
}

static int pb_solve_dev_impl(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                 const int32_t *d_tri, int64_t n_charges, const double *d_pos, const double *d_q,
                 const pb_params *p, double *d_phi, double *d_dphi, pb_info *info)
{
    const double t0 = now_s();
    TRY(enter(c));
    const int st = solve_dev(c, n_vert, n_tri, d_vert, d_tri, n_charges, d_pos, d_q, p, d_phi,
                             d_dphi, info);
    if (info && st >= 0)
        info->seconds = now_s() - t0;
    return st;
}


int pb_geometry(pb_ctx *c, const pb_surface *s, double *cen, double *nrm, double *area)
{
    return leave(c, guarded(c, [&] { return pb_geometry_impl(c, s, cen, nrm, area); }));
}

int pb_source(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p, double *b)
{
    return leave(c, guarded(c, [&] { return pb_source_impl(c, s, q, p, b); }));
}

int pb_matvec(pb_ctx *c, const pb_surface *s, const pb_params *p, const double *x, double *y,
              int transpose, int precision)
{
    return leave(c, guarded(c, [&] {
        return pb_matvec_impl(c, s, p, x, y, transpose, precision);
    }));
}

int pb_solve_tree(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
                  double theta, int order, int leaf_size, double *phi, double *dphi,
                  pb_info *info)
{
    return leave(c, guarded(c, [&] {
        return pb_solve_tree_impl(c, s, q, p, theta, order, leaf_size, phi, dphi, info);
    }));
}

int pb_matvec_tree(pb_ctx *c, const pb_surface *s, const pb_params *p, double theta, int order,
                   int leaf_size, const double *x, double *y, int64_t *counts)
{
    return leave(c, guarded(c, [&] {
        return pb_matvec_tree_impl(c, s, p, theta, order, leaf_size, x, y, counts);
    }));
}

int pb_matvec_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, const pb_params *p, const double *d_x, double *d_y,
                  int transpose, int precision)
{
    return leave(c, guarded(c, [&] {
        return pb_matvec_dev_impl(c, n_vert, n_tri, d_vert, d_tri, p, d_x, d_y, transpose,
                                  precision);
    }));
}

int pb_matvec_dev_noalloc(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                          const int32_t *d_tri, const pb_params *p, const double *d_x,
                          double *d_y, int transpose, int precision)
{
    return leave(c, guarded(c, [&]() -> int {
        TRY(enter(c));
        return matvec_noalloc(c, n_vert, n_tri, d_vert, d_tri, p, d_x, d_y, transpose ? 1 : 0,
                              precision);
    }));
}

int pb_source_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, int64_t n_charges, const double *d_pos, const double *d_q,
                  const pb_params *p, double *d_b)
{
    return leave(c, guarded(c, [&] {
        return pb_source_dev_impl(c, n_vert, n_tri, d_vert, d_tri, n_charges, d_pos, d_q, p,
                                  d_b);
    }));
}

int pb_energy_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, int64_t n_charges, const double *d_pos, const double *d_q,
                  const pb_params *p, const double *d_phi, const double *d_dphi, double *e_solv)
{
    return leave(c, guarded(c, [&] {
        return pb_energy_dev_impl(c, n_vert, n_tri, d_vert, d_tri, n_charges, d_pos, d_q, p,
                                  d_phi, d_dphi, e_solv);
    }));
}

int pb_energy(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
              const double *phi, const double *dphi, double *e_solv)
{
    return leave(c, guarded(c, [&] { return pb_energy_impl(c, s, q, p, phi, dphi, e_solv); }));
}

int pb_solve(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
             double *phi, double *dphi, pb_info *info)
{
    return leave(c, guarded(c, [&] { return pb_solve_impl(c, s, q, p, phi, dphi, info); }));
}

int pb_solve_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                 const int32_t *d_tri, int64_t n_charges, const double *d_pos, const double *d_q,
                 const pb_params *p, double *d_phi, double *d_dphi, pb_info *info)
{
    return leave(c, guarded(c, [&] {
        return pb_solve_dev_impl(c, n_vert, n_tri, d_vert, d_tri, n_charges, d_pos, d_q, p, d_phi,
                                 d_dphi, info);
    }));
}

int pb_forces(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
              double *dE_dpos, double *dE_dq, pb_info *info)
{
    return leave(c, guarded(c, [&] { return pb_forces_impl(c, s, q, p, dE_dpos, dE_dq, info); }));
}

int pb_forces_dev(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, int64_t n_charges, const double *d_pos,
                  const double *d_q, const pb_params *p, double *d_dE_dpos, double *d_dE_dq,
                  pb_info *info)
{
    return leave(c, guarded(c, [&] {
        return pb_forces_dev_impl(c, n_vert, n_tri, d_vert, d_tri, n_charges, d_pos, d_q, p,
                                  d_dE_dpos, d_dE_dq, info);
    }));
}

static int pb_potential_impl(pb_ctx *c, const pb_surface *s, const pb_charges *q,
                             const pb_params *p, const double *phi, const double *dphi,
                             int64_t n_points, const double *points, double *reaction,
                             double *total)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!phi || !dphi || !points || n_points <= 0)
        return fail(c, PB_ERR_ARG, "phi, dphi or points missing");
    const double *dv, *dp, *dq;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(upload_charges(c, q, &dp, &dq));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    const Geo &g = c->g;
    const int64_t n = s->n_tri;
    TRY(ensure(c, c->io_x, sizeof(double) * (2 * n + 3 * n_points)));
    double *dx = as<double>(c->io_x), *dpts = dx + 2 * n;
    HIPCHK(hipMemcpyAsync(dx, phi, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dx + n, dphi, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dpts, points, sizeof(double) * 3 * n_points, hipMemcpyHostToDevice,
                          c->stream));
    const Sweep sw = plan_sweep(n_points, g.npad, TARGET_WAVES);
    const int64_t ncpad = (int64_t)sw.n_tblocks * TPB;
    TRY(ensure(c, c->chg_part, sizeof(double) * sw.n_chunks * ncpad));
    TRY(ensure(c, c->chg_per, sizeof(double) * ncpad));
    TRY(ensure(c, c->src64, sizeof(double) * 8 * g.npad));
    TRY(ensure(c, c->io_y, sizeof(double) * 2 * n_points));
    double *reac = as<double>(c->io_y), *coul = reac + n_points;
    launch_pack_f64(c->stream, g, dx, as<double>(c->src64), 0);
    LAUNCHCHK();
    launch_charge_pairs(c->stream, g, as<double>(c->src64), n_points, dpts, sw, pair_params(c, p),
                        0, as<double>(c->chg_part), ncpad);
    LAUNCHCHK();
    launch_charge_finish(c->stream, as<double>(c->chg_part), sw.n_chunks, n_points, ncpad, nullptr,
                         1.0, reac, nullptr);
    LAUNCHCHK();
    launch_point_coulomb(c->stream, n_points, dpts, q->n, dp, dq,
                         1.0 / (4.0 * M_PI * p->eps_in), 0, coul);
    LAUNCHCHK();
    std::vector<double> hr(n_points), hc(n_points);
    HIPCHK(hipMemcpyAsync(hr.data(), reac, sizeof(double) * n_points, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(hc.data(), coul, sizeof(double) * n_points, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int64_t k = 0; k < n_points; ++k) {
        const double r = hr[k] / (4.0 * M_PI);   // the sweep sums 4 pi K
        if (reaction)
            reaction[k] = r;
        if (total)
            total[k] = r + hc[k];
    }
    return PB_OK;
}

static int pb_coulomb_energy_impl(pb_ctx *c, const pb_charges *q, const pb_params *p,
                                  double *e_coul)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!e_coul)
        return fail(c, PB_ERR_ARG, "e_coul is NULL");
    const double *dp, *dq;
    TRY(upload_charges(c, q, &dp, &dq));
    TRY(ensure(c, c->chg_per, sizeof(double) * q->n));
    TRY(ensure(c, c->small, sizeof(double) * HSMALL));
    launch_point_coulomb(c->stream, q->n, dp, q->n, dp, dq, 1.0 / p->eps_in, 1,
                         as<double>(c->chg_per));
    LAUNCHCHK();
    const int slot = HSMALL - 4;
    launch_weighted_total(c->stream, as<double>(c->chg_per), dq, q->n, 0.5 * C_UNITS,
                          as<double>(c->small) + slot);
    LAUNCHCHK();
    TRY(fetch_small(c, slot, 1));
    *e_coul = c->hsmall[slot];
    return PB_OK;
}

int pb_potential(pb_ctx *c, const pb_surface *s, const pb_charges *q, const pb_params *p,
                 const double *phi, const double *dphi, int64_t n_points, const double *points,
                 double *reaction, double *total)
{
    return leave(c, guarded(c, [&] {
        return pb_potential_impl(c, s, q, p, phi, dphi, n_points, points, reaction, total);
    }));
}

int pb_coulomb_energy(pb_ctx *c, const pb_charges *q, const pb_params *p, double *e_coul)
{
    return leave(c, guarded(c, [&] { return pb_coulomb_energy_impl(c, q, p, e_coul); }));
}

static int pb_precond_leaves_impl(pb_ctx *c, const pb_surface *s, int leaf, int32_t *perm,
                                  int32_t *leaf_start, int64_t *n_leaves)
{
    TRY(enter(c));
    if (!perm || !leaf_start || !n_leaves)
        return fail(c, PB_ERR_ARG, "output arrays are NULL");
    if (leaf < 1 || leaf > PC_MAX_LEAF)
        return fail(c, PB_ERR_ARG, "leaf must be in [1, %d]", PC_MAX_LEAF);
    const double *dv;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    pb_params p{};
    p.eps_in = 1.0;
    p.eps_out = 1.0;
    p.precond_leaf = leaf;
    TRY(setup_precond(c, &p));
    const int64_t L = c->pc_leaves;
    HIPCHK(hipMemcpyAsync(perm, c->pc_perm, sizeof(int32_t) * s->n_tri, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(leaf_start, c->pc_start, sizeof(int32_t) * (L + 1),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *n_leaves = L;
    return PB_OK;
}

static int pb_precond_apply_impl(pb_ctx *c, const pb_surface *s, const pb_params *p,
                                 const double *x, double *y, int transpose)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    if (!x || !y)
        return fail(c, PB_ERR_ARG, "x or y is NULL");
    if (p->precond_leaf < 1 || p->precond_leaf > PC_MAX_LEAF)
        return fail(c, PB_ERR_ARG, "precond_leaf must be in [1, %d]", PC_MAX_LEAF);
    const double *dv;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    TRY(setup_precond(c, p));
    const int64_t n2 = 2 * s->n_tri;
    TRY(ensure(c, c->io_x, sizeof(double) * n2));
    TRY(ensure(c, c->io_y, sizeof(double) * n2));
    HIPCHK(hipMemcpyAsync(c->io_x.p, x, sizeof(double) * n2, hipMemcpyHostToDevice, c->stream));
    TRY(pc_apply(c, transpose ? 1 : 0, as<double>(c->io_x), as<double>(c->io_y)));
    HIPCHK(hipMemcpyAsync(y, c->io_y.p, sizeof(double) * n2, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

int pb_precond_leaves(pb_ctx *c, const pb_surface *s, int leaf, int32_t *perm,
                      int32_t *leaf_start, int64_t *n_leaves)
{
    return leave(c, guarded(c, [&] {
        return pb_precond_leaves_impl(c, s, leaf, perm, leaf_start, n_leaves);
    }));
}

int pb_precond_apply(pb_ctx *c, const pb_surface *s, const pb_params *p, const double *x,
                     double *y, int transpose)
{
    return leave(c, guarded(c, [&] { return pb_precond_apply_impl(c, s, p, x, y, transpose); }));
}

int pb_set_sweep_config(pb_ctx *c, int targets_per_thread, int target_waves)
{
    if (!c)
        return PB_ERR_ARG;
    if (targets_per_thread != 0 && targets_per_thread != 1 && targets_per_thread != 2 &&
        targets_per_thread != PB_SWEEP_PAIRWISE && targets_per_thread != PB_SWEEP_BANDED)
        return fail(c, PB_ERR_ARG,
                    "sweep kind must be 1, 2, PB_SWEEP_PAIRWISE or PB_SWEEP_BANDED");
    if (target_waves < 0 || target_waves > (1 << 22))
        return fail(c, PB_ERR_ARG, "target_waves out of range");
    if (targets_per_thread)
        c->f32_tpt = targets_per_thread;
    if (target_waves)
        c->f32_waves = target_waves;
    return PB_OK;
}

int pb_set_fp64_sweep(pb_ctx *c, int kind)
{
    if (!c)
        return PB_ERR_ARG;
    if (kind != 0 && kind != 1 && kind != PB_SWEEP_PAIRWISE)
        return fail(c, PB_ERR_ARG, "FP64 sweep kind must be 1 or PB_SWEEP_PAIRWISE");
    if (kind)
        c->f64_kind = kind;
    return PB_OK;
}

int pb_get_fp64_sweep(pb_ctx *c, int *kind)
{
    if (!c)
        return PB_ERR_ARG;
    if (kind)
        *kind = c->f64_kind;
    return PB_OK;
}

int pb_get_sweep_config(pb_ctx *c, int *targets_per_thread, int *target_waves)
{
    if (!c)
        return PB_ERR_ARG;
    if (targets_per_thread)
        *targets_per_thread = c->f32_tpt;
    if (target_waves)
        *target_waves = c->f32_waves;
    return PB_OK;
}

static int pb_autotune_impl(pb_ctx *c, const pb_surface *s, const pb_params *p, int *best_tpt,
                            int *best_waves)
{
    TRY(enter(c));
    TRY(check_params(c, p, false));
    const double *dv;
    const int32_t *dt;
    TRY(upload_surface(c, s, &dv, &dt));
    TRY(setup_geometry(c, s->n_vert, s->n_tri, dv, dt));
    const int64_t n2 = 2 * c->g.n;
    TRY(ensure(c, c->io_x, sizeof(double) * n2));
    TRY(ensure(c, c->io_y, sizeof(double) * n2));
    launch_fill(c->stream, as<double>(c->io_x), 1.0, n2);
    LAUNCHCHK();
    static const int tpts[] = {PB_SWEEP_PAIRWISE, PB_SWEEP_BANDED, 1, 2};
    static const int waves[] = {8192, 16384, 32768, 65536, 131072, 262144};
    hipEvent_t e0 = pool_event(c, 0), e1 = pool_event(c, 1);
    if (!e0 || !e1)
        return fail(c, PB_ERR_HIP, "hipEventCreate failed");
    const bool prof = c->prof_on;
    c->prof_on = false;
    float best = 0.f;
    int bt = c->f32_tpt, bw = c->f32_waves;
    for (int tp : tpts) {
        for (int wv : waves) {
            c->f32_tpt = tp;
            c->f32_waves = wv;
            int rc = apply(c, p, PB_FP32_IR, 0, as<double>(c->io_x), as<double>(c->io_y));
            if (rc < 0) {
                c->prof_on = prof;
                return rc;
            }
            HIPCHK(hipEventRecord(e0, c->stream));
            for (int rep = 0; rep < 2; ++rep)
                TRY(apply(c, p, PB_FP32_IR, 0, as<double>(c->io_x), as<double>(c->io_y)));
            HIPCHK(hipEventRecord(e1, c->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (best == 0.f || ms < best) {
                best = ms;
                bt = tp;
                bw = wv;
            }
        }
    }
    c->prof_on = prof;
    c->f32_tpt = bt;
    c->f32_waves = bw;
    if (best_tpt)
        *best_tpt = bt;
    if (best_waves)
        *best_waves = bw;
    return PB_OK;
}

int pb_autotune(pb_ctx *c, const pb_surface *s, const pb_params *p, int *best_tpt,
                int *best_waves)
{
    return leave(c, guarded(c, [&] { return pb_autotune_impl(c, s, p, best_tpt, best_waves); }));
}

static int pb_solve_batch_impl(pb_ctx *c, int32_t n_sys, const pb_surface *surf,
                               const pb_charges *chg, const pb_params *p, double *e_solv,
                               double *dE_dpos, double *dE_dq, pb_info *info)
{
    const double t0 = now_s();
    TRY(enter(c));
    TRY(check_params(c, p, true));
    const int want = (dE_dpos != nullptr) || (dE_dq != nullptr);
    const int st = batch_solve(c, n_sys, surf, chg, p, want, e_solv, dE_dpos, dE_dq, info);
    if (info && st >= 0) {
        const double dt = now_s() - t0;
        for (int b = 0; b < n_sys; ++b)
            info[b].seconds = dt;
    }
    return st;
}

int pb_solve_batch(pb_ctx *c, int32_t n_sys, const pb_surface *surf, const pb_charges *chg,
                   const pb_params *p, double *e_solv, double *dE_dpos, double *dE_dq,
                   pb_info *info)
{
    return leave(c, guarded(c, [&] {
        return pb_solve_batch_impl(c, n_sys, surf, chg, p, e_solv, dE_dpos, dE_dq, info);
    }));
}

static int pb_solve_batch_dev_impl(pb_ctx *c, int32_t n_sys, const pb_surface *surf,
                                   const pb_charges *chg, const pb_params *p, double *e_solv,
                                   double *d_dE_dpos, double *d_dE_dq, pb_info *info)
{
    const double t0 = now_s();
    TRY(enter(c));
    TRY(check_params(c, p, true));
    const int want = (d_dE_dpos != nullptr) || (d_dE_dq != nullptr);
    const int st = batch_solve(c, n_sys, surf, chg, p, want, e_solv, d_dE_dpos, d_dE_dq, info,
                               nullptr, true);
    if (info && st >= 0) {
        const double dt = now_s() - t0;
        for (int b = 0; b < n_sys; ++b)
            info[b].seconds = dt;
    }
    return st;
}

int pb_solve_batch_dev(pb_ctx *c, int32_t n_sys, const pb_surface *surf, const pb_charges *chg,
                       const pb_params *p, double *e_solv, double *d_dE_dpos, double *d_dE_dq,
                       pb_info *info)
{
    return leave(c, guarded(c, [&] {
        return pb_solve_batch_dev_impl(c, n_sys, surf, chg, p, e_solv, d_dE_dpos, d_dE_dq, info);
    }));
}

static int pb_autotune_batch_impl(pb_ctx *c, int32_t n_sys, const pb_surface *surf,
                                  const pb_charges *chg, const pb_params *p, int *best_kind,
                                  int *best_tiles)
{
    TRY(enter(c));
    TRY(check_params(c, p, true));
    BatchTune tn;
    const int tiles[] = {2, 4, 8, 16, 32};
    for (int t : tiles) {
        tn.kind[tn.n] = PB_SWEEP_PAIRWISE;
        tn.tiles[tn.n++] = t;
    }
    tn.kind[tn.n] = 1;   // per-target sweep
    tn.tiles[tn.n++] = 0;
    TRY(batch_solve(c, n_sys, surf, chg, p, 0, nullptr, nullptr, nullptr, nullptr, &tn));
    if (best_kind)
        *best_kind = c->f32_tpt;
    if (best_tiles)
        *best_tiles = c->b_sym_tiles;
    return PB_OK;
}

int pb_autotune_batch(pb_ctx *c, int32_t n_sys, const pb_surface *surf, const pb_charges *chg,
                      const pb_params *p, int *best_kind, int *best_tiles)
{
    return leave(c, guarded(c, [&] {
        return pb_autotune_batch_impl(c, n_sys, surf, chg, p, best_kind, best_tiles);
    }));
}

int pb_set_batch_tiles(pb_ctx *c, int tiles)
{
    if (!c)
        return PB_ERR_ARG;
    if (tiles < 0 || tiles > 1024)
        return fail(c, PB_ERR_ARG, "batch tiles per item must be in [1, 1024] (0: unchanged)");
    if (tiles > 0)
        c->b_sym_tiles = tiles;
    return PB_OK;
}

int pb_get_batch_tiles(pb_ctx *c, int *tiles)
{
    if (!c || !tiles)
        return PB_ERR_ARG;
    *tiles = c->b_sym_tiles;
    return PB_OK;
}

int pb_set_memory_limit(pb_ctx *c, int64_t bytes)
{
    if (!c)
        return PB_ERR_ARG;
    if (bytes < 0)
        return fail(c, PB_ERR_ARG, "memory limit must be >= 0");
    c->mem_limit = (size_t)bytes;
    return PB_OK;
}

int pb_get_memory_used(pb_ctx *c, int64_t *bytes)
{
    if (!c || !bytes)
        return PB_ERR_ARG;
    *bytes = (int64_t)c->mem_used;
    return PB_OK;
}

int pb_profile_enable(pb_ctx *c, int enable)
{
    if (!c)
        return PB_ERR_ARG;
    c->prof_on = enable != 0;
    return PB_OK;
}

int pb_profile_reset(pb_ctx *c)
{
    if (!c)
        return PB_ERR_ARG;
    for (int k = 0; k < PB_KERNEL_COUNT; ++k) {
        c->prof_launches[k] = 0;
        c->prof_ms[k] = 0.0;
        c->prof_pairs[k] = 0.0;
    }
    c->marks.clear();
    return PB_OK;
}

int pb_profile_read(pb_ctx *c, int kernel, int64_t *launches, double *total_ms, double *pairs)
{
    if (!c)
        return PB_ERR_ARG;
    if (kernel < 0 || kernel >= PB_KERNEL_COUNT)
        return fail(c, PB_ERR_ARG, "kernel id %d out of range", kernel);
    if (launches)
        *launches = c->prof_launches[kernel];
    if (total_ms)
        *total_ms = c->prof_ms[kernel];
    if (pairs)
        *pairs = c->prof_pairs[kernel];
    return PB_OK;
}

static int pb_eval_pair_math_impl(pb_ctx *c, int64_t n, const double *x, const double *y,
                                  double *exp_out, double *rsqrt_out)
{
    TRY(enter(c));
    if (n < 0 || n > PB_PAIR_MATH_MAX)
        return fail(c, PB_ERR_ARG, "n = %lld outside [0, %d]", (long long)n, PB_PAIR_MATH_MAX);
    if (n == 0)
        return PB_OK;
    if (!x || !y || !exp_out || !rsqrt_out)
        return fail(c, PB_ERR_ARG, "an argument or result array is NULL");
    for (int64_t k = 0; k < n; ++k) {
        if (!(x[k] >= 0.0 && x[k] <= PB_PAIR_MATH_XMAX))
            return fail(c, PB_ERR_ARG, "x[%lld] = %g outside [0, %g]", (long long)k, x[k],
                        PB_PAIR_MATH_XMAX);
        if (!(y[k] >= PB_PAIR_MATH_YMIN && y[k] <= PB_PAIR_MATH_YMAX))
            return fail(c, PB_ERR_ARG, "y[%lld] = %g outside [%g, %g]", (long long)k, y[k],
                        PB_PAIR_MATH_YMIN, PB_PAIR_MATH_YMAX);
    }
    const size_t bytes = sizeof(double) * (size_t)n;
    TRY(ensure(c, c->io_x, 2 * bytes));
    TRY(ensure(c, c->io_y, 2 * bytes));
    double *dx = as<double>(c->io_x), *dy = as<double>(c->io_y);
    HIPCHK(hipMemcpyAsync(dx, x, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dx + n, y, bytes, hipMemcpyHostToDevice, c->stream));
    launch_eval_pair_math(c->stream, n, dx, dx + n, dy, dy + n);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(exp_out, dy, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(rsqrt_out, dy + n, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

int pb_eval_pair_math(pb_ctx *c, int64_t n, const double *x, const double *y, double *exp_out,
                      double *rsqrt_out)
{
    return leave(c, guarded(c, [&] {
        return pb_eval_pair_math_impl(c, n, x, y, exp_out, rsqrt_out);
    }));
}

int pb_probe_valu(pb_ctx *c, int kind, int64_t *lane_ops)
{
    if (!c || !lane_ops)
        return PB_ERR_ARG;
    if (kind < PB_PROBE_FMA_F32 || kind > PB_PROBE_EXP_F32)
        return fail(c, PB_ERR_ARG, "probe kind %d out of range", kind);
    HIPCHK(hipSetDevice(c->device));
    TRY(ensure(c, c->probe_out, sizeof(double) * (size_t)PROBE_THREADS));
    *lane_ops = launch_probe_valu(c->stream, kind, as<double>(c->probe_out));
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->stream));
    return PB_OK;
}

}  // extern "C"
