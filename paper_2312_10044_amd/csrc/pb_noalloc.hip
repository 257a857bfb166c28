// pb_matvec_dev_noalloc: the matvec of eqs. eqbim_5/eqbim_6 (and its
// transpose) on device-resident inputs with no device allocation, for callers
// that cannot allocate (code under stream capture, tight serving loops).
//
// Every buffer the kernels need beyond the caller's inputs and outputs (the
// collocation geometry, its validation reductions, the coincident-centroid
// table, the packed source stream and the chunk partials of the per-target
// sweep) lives in one file-scope device array, `scratch`, of NA_DOUBLES
// doubles (about 14 MB), which each GPU the library runs on holds until the
// process ends.  Host code never uses the array's name as an address: the
// device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress when a context is created there (noalloc_init), and the
// launches take that pointer.  All calls on one GPU share its copy; every
// kernel writes what it later reads (the geometry and partials entirely, the
// hash table is cleared first), so nothing carries over between calls, but
// calls that overlap in time on one GPU race.  Sizes: n_tri <= NA_MAX_TRI.
#include "../../include/pbsolve.h"
#include "pb_ctx.h"
#include "pb_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

namespace pbk {

namespace {

constexpr int64_t NA_MAX_TRI = 32768;          // largest surface (a multiple of PADN)
constexpr int NA_MAX_CHUNKS = 16;              // source chunks of the per-target sweep
constexpr int NA_MAX_GEO_BLOCKS = 1024;        // geometry_blocks() never exceeds this
constexpr int64_t NA_DUP_CAP = 65536;          // dup_table_size(NA_MAX_TRI)
// layout, in doubles
constexpr int64_t NA_GEO = 0;                                      // NGEO * NA_MAX_TRI
constexpr int64_t NA_GPART = NA_GEO + NGEO * NA_MAX_TRI;           // GEO_RED * blocks
constexpr int64_t NA_SMALL = NA_GPART + GEO_RED * NA_MAX_GEO_BLOCKS;
constexpr int64_t NA_SRC = NA_SMALL + 64;                          // 8 values per source
constexpr int64_t NA_PART = NA_SRC + 8 * NA_MAX_TRI;               // 2 * chunks * npad
constexpr int64_t NA_DUP = NA_PART + 2 * NA_MAX_CHUNKS * NA_MAX_TRI;   // int32 table
constexpr int64_t NA_DOUBLES = NA_DUP + (NA_DUP_CAP + 2 + 1) / 2;

__device__ __align__(256) double scratch[NA_DOUBLES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
double *na_ptr[NA_MAX_DEVICES] = {};   // device address of `scratch`, per GPU

}  // namespace

int noalloc_init(int device)
{
    if (device < 0 || device >= NA_MAX_DEVICES)
        return PB_ERR_ARG;
    std::lock_guard<std::mutex> lk(na_mutex);
    if (na_ptr[device])
        return PB_OK;
    void *p = nullptr;
    // the calling thread has `device` current (pb_create set it)
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return PB_ERR_HIP;
    }
    na_ptr[device] = static_cast<double *>(p);
    return PB_OK;
}

int matvec_noalloc(pb_ctx *c, int64_t n_vert, int64_t n_tri, const double *d_vert,
                   const int32_t *d_tri, const pb_params *p, const double *d_x, double *d_y,
                   int transpose, int precision)
{
    if (!p)
        return fail(c, PB_ERR_ARG, "params is NULL");
    if (!(p->eps_in > 0.0) || !(p->eps_out > 0.0) || !std::isfinite(p->eps_in) ||
        !std::isfinite(p->eps_out))
        return fail(c, PB_ERR_ARG, "eps_in and eps_out must be finite and > 0");
    if (!(p->kappa >= 0.0) || !(p->kappa <= KAPPA_MAX))
        return fail(c, PB_ERR_ARG, "kappa must lie in [0, %g] 1/A", KAPPA_MAX);
    if (precision != PB_FP64 && precision != PB_FP32_IR)
        return fail(c, PB_ERR_ARG, "precision must be PB_FP64 or PB_FP32_IR");
    if (!d_vert || !d_tri || !d_x || !d_y)
        return fail(c, PB_ERR_ARG, "a device array is NULL");
    if (n_tri < 1 || n_vert < 3)
        return fail(c, PB_ERR_ARG, "need n_tri > 0 and n_vert >= 3");
    if (n_tri > NA_MAX_TRI)
        return fail(c, PB_ERR_ARG,
                    "pb_matvec_dev_noalloc takes at most %lld triangles (got %lld): its scratch "
                    "is a fixed device array; use pb_matvec_dev",
                    (long long)NA_MAX_TRI, (long long)n_tri);
    double *base = (c->device >= 0 && c->device < NA_MAX_DEVICES) ? na_ptr[c->device] : nullptr;
    if (!base)
        return fail(c, PB_ERR_HIP, "no-allocation scratch of device %d is not set up",
                    c->device);
    hipStream_t s = c->stream;
    const int64_t npad = round_up(n_tri, PADN);
    double *geo = base + NA_GEO, *gpart = base + NA_GPART, *small = base + NA_SMALL;
    int32_t *dup = reinterpret_cast<int32_t *>(base + NA_DUP);
    const int nblk = geometry_blocks(npad);
    const int64_t cap = dup_table_size(n_tri);
    if (nblk > NA_MAX_GEO_BLOCKS || cap > NA_DUP_CAP)
        return fail(c, PB_ERR_ARG, "internal: no-allocation layout too small");
    // step 1 with validation, as for every entry point
    launch_geometry(s, n_vert, n_tri, d_vert, d_tri, geo, npad, npad, gpart, nblk);
    LAUNCHCHK();
    launch_reduce_cols(s, gpart, nblk, GEO_RED, small);
    LAUNCHCHK();
    launch_dup_check(s, geo, n_tri, npad, dup, cap);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(c->hsmall, small, sizeof(double) * GEO_RED, hipMemcpyDeviceToHost, s));
    int32_t *hdup = reinterpret_cast<int32_t *>(c->hsmall + HSMALL_DUP);
    HIPCHK(hipMemcpyAsync(hdup, dup + cap, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double *r = c->hsmall;
    if (r[0] != 0.0)
        return fail(c, PB_ERR_GEOMETRY,
                    "%.0f triangle(s) with an out-of-range index, a non-finite vertex or zero area",
                    r[0]);
    if (r[6] != 0.0)
        return fail(c, PB_ERR_GEOMETRY,
                    "%.0f triangle(s) with a centroid coordinate beyond %g A", r[6], COORD_MAX);
    if (hdup[1] != 0)
        return fail(c, PB_ERR_GEOMETRY,
                    "triangle %d shares its centroid with another triangle: collocation points "
                    "must be distinct",
                    hdup[0]);
    if (!(r[1] > 0.0))
        return fail(c, PB_ERR_GEOMETRY,
                    "enclosed volume %.6g <= 0: triangles must be counter-clockwise seen from "
                    "outside",
                    r[1] / 6.0);
    const Geo g{geo, n_tri, npad};
    PairParams pp;
    pp.eps = p->eps_out / p->eps_in;
    pp.kappa = p->kappa;
    pp.cx = r[2] / (double)n_tri;
    pp.cy = r[3] / (double)n_tri;
    pp.cz = r[4] / (double)n_tri;
    pp.sigma = f32_sigma(p->kappa, 1.0 / std::sqrt(r[5] / (2.0 * TWO_PI)));
    // per-target sweep, its source range cut into at most NA_MAX_CHUNKS chunks
    const bool fwd32 = precision == PB_FP32_IR && !transpose;
    Sweep sw = plan_sweep(npad, npad, TARGET_WAVES, 1);
    if (sw.n_chunks > NA_MAX_CHUNKS) {
        sw.tiles_per_chunk = (sw.n_tiles + NA_MAX_CHUNKS - 1) / NA_MAX_CHUNKS;
        sw.n_chunks = (sw.n_tiles + sw.tiles_per_chunk - 1) / sw.tiles_per_chunk;
    }
    double *part = base + NA_PART;
    const double eps = pp.eps;
    double scale1 = 1.0, scale2 = 1.0;
    if (fwd32) {
        float *src = reinterpret_cast<float *>(base + NA_SRC);
        launch_pack_f32(s, g, d_x, src, 2, pp.cx, pp.cy, pp.cz, eps, pp.sigma);
        LAUNCHCHK();
        launch_pairs_f32_fwd(s, g, src, sw, pp, 1, part);
        scale1 = eps * pp.sigma * pp.sigma;
        scale2 = pp.sigma * pp.sigma * pp.sigma;
    } else if (precision == PB_FP32_IR) {
        float *src = reinterpret_cast<float *>(base + NA_SRC);
        launch_pack_f32(s, g, d_x, src, 1, pp.cx, pp.cy, pp.cz, eps, 1.0);
        LAUNCHCHK();
        launch_pairs_f32(s, g, src, sw, pp, 1, part);
    } else {
        double *src = base + NA_SRC;
        launch_pack_f64(s, g, d_x, src, transpose ? 1 : 0);
        LAUNCHCHK();
        launch_pairs_f64(s, g, src, sw, pp, transpose ? 1 : 0, part);
    }
    LAUNCHCHK();
    launch_matvec_finish(s, g, part, sw.n_chunks, d_x, 0.5 * (1.0 + eps), 0.5 * (1.0 + 1.0 / eps),
                         transpose ? 1 : 0, scale1, scale2, d_y);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
    return PB_OK;
}

}  // namespace pbk
