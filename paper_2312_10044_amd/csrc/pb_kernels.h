// Internal interface between the HIP kernels (pb_kernels.hip) and the host
// driver (pb_capi.hip).  Not part of the public ABI.
#pragma once

#include "pb_host.h"

#include <hip/hip_runtime.h>

#include <vector>
#include <cstdint>

namespace pbk {

constexpr int TPB = 256;        // threads per block of every pair kernel
static_assert(TILE == TPB, "a tile is one block's worth of targets");
constexpr int NGEO = 7;         // cx, cy, cz, nx, ny, nz, area
constexpr int GEO_RED = 7;      // bad, 6*volume, sum cx, sum cy, sum cz, sum area, far
constexpr double COORD_MAX = 1.0e5;   // |centroid coordinate| bound, A (padding sits at 2e6)
constexpr double KAPPA_MAX = 100.0;   // 1/A: kappa r stays < 1.4e9 for every padded pair
constexpr int MAX_RESTART = 64;
constexpr int PADN = 512;       // collocation arrays are padded to a multiple of this
constexpr int PC_MAX_LEAF = 100; // largest preconditioner leaf (N0 of Sec. 2.2.4's runs)

// Device-side collocation geometry, SoA: array k at g + k * npad.
struct Geo {
    const double *g;
    int64_t n;      // triangles
    int64_t npad;   // n rounded up to a multiple of PADN
};

struct PairParams {
    double eps;         // eps_out / eps_in
    double kappa;
    double cx, cy, cz;  // origin subtracted from positions before FP32 arithmetic
    double sigma;       // FP32 length unit: positions are multiplied by it (f32_sigma)
};

// Launch shape of one pair sweep: targets in blocks of TPB, sources split
// into n_chunks contiguous ranges of tiles_per_chunk tiles.
struct Sweep {
    int n_tblocks;
    int n_tiles;
    int n_chunks;
    int tiles_per_chunk;
};

// tpt = targets per thread (blocks cover TPB * tpt targets).
Sweep plan_sweep(int64_t n_targets, int64_t n_sources, int target_waves, int tpt = 1);

// geometry + per-block partial reductions (GEO_RED columns x nblk)
int geometry_blocks(int64_t n_tri);
// Writes entries [0, npad) of the seven arrays g + k * ld.
void launch_geometry(hipStream_t s, int64_t n_vert, int64_t n_tri, const double *vert,
                     const int32_t *tri, double *g, int64_t npad, int64_t ld, double *part,
                     int nblk);

// Packed source stream: 8 values per source (x, y, z, w, mx, my, mz, pad).
// mode 0 (forward): w = a_j psi_j, m = a_j phi_j n_j.
// mode 1 (transpose): w = l1_j, m = l2_j n_j.
// mode 2 (FP32 forward, reduced form): w = (1-1/eps) a psi / sigma,
//        m = -3 a phi n, pad = -a psi / (eps sigma), positions times sigma.
void launch_pack_f64(hipStream_t s, const Geo &geo, const double *x, double *src, int mode);
void launch_pack_f32(hipStream_t s, const Geo &geo, const double *x, float *src, int mode,
                     double cx, double cy, double cz, double eps, double sigma);
// Length unit of the reduced FP32 form: positions are multiplied by sigma.
// sigma = kappa makes kappa r the distance itself (the SCALED kernels).  When
// kappa is below sigma_min, the inverse of the mesh's own length scale (and at
// kappa = 0), the unit is 1/sigma_min and the kernels take kappa / sigma:
// bounding sigma from below keeps (sigma r)^-3 of the nearest pairs far from
// FP32 overflow however small kappa is.  Row 1 of the sweep carries a factor
// sigma^2 and row 2 a factor sigma^3.
inline double f32_sigma(double kappa, double sigma_min)
{
    return kappa >= sigma_min ? kappa : sigma_min;
}
inline bool f32_scaled(const PairParams &pp) { return pp.kappa > 0.0 && pp.sigma == pp.kappa; }

// Exact coincidence of collocation points: the singular term is skipped by
// index (j = i), so two triangles with the same centroid would meet at r = 0.
// tab: cap int32 slots (cap a power of two >= 2 n) followed by out[2] =
// {smallest index that shares its centroid with another point (INT32_MAX if
// none), number of such coincidences}; both are independent of scheduling.
// Triangles of zero area (rejected ones) are skipped.
void launch_dup_check(hipStream_t s, const double *g, int64_t n, int64_t ld, int32_t *tab,
                      int64_t cap);

// Pair sweep of the matvec: part[(o * n_chunks + c) * npad + i], o in {0,1}.
void launch_pairs_f64(hipStream_t s, const Geo &geo, const double *src, const Sweep &sw,
                      const PairParams &pp, int transpose, double *part);
void launch_pairs_f32(hipStream_t s, const Geo &geo, const float *src, const Sweep &sw,
                      const PairParams &pp, int transpose, double *part);
// FP32 forward sweep (mode-2 stream), tpt in {1, 2} targets per thread.
void launch_pairs_f32_fwd(hipStream_t s, const Geo &geo, const float *src, const Sweep &sw,
                          const PairParams &pp, int tpt, double *part);
// Pairwise FP32 forward sweep (each unordered pair once).  Work items
// (I, J0, J1, slot): target tile I against source tiles J0..J1-1 (J0 >= I; the
// tile J = I runs forward only).  Row sums of item k land in
// rowpart[k][2][TILE] (FP64); the contributions of off-diagonal tile pair
// (I, J) to the rows of tile J land in colpart[pair_index(I, J)][2][TILE]
// (FP32).  row_start[K]..row_start[K+1] are the item slots of target tile K.
// SymPlan and plan_sym (the work items) are host code, in pb_host.h.
// Upper-triangle index of tile pair (I, J), I < J < T.
__host__ __device__ inline int64_t sym_pair_index(int64_t I, int64_t J, int64_t T)
{
    return I * T - I * (I + 1) / 2 + (J - I - 1);
}
// Banded pairwise FP32 sweep (sweep kind PB_SWEEP_BANDED): blocks of
// BAND_WAVES waves hold BAND_MT target tiles (a macro tile); a work item is a
// band of macro tiles [m0, m1) against a run of source tiles [j0, j1).  Its
// records (2 x TILE floats each) hold the rows of each target tile I of the
// band over the run (rslot + I - BAND_MT m0, written when j1 > I) and the
// column sums of each source tile J of the run over the band (cslot + J - j0).
// rec_start[K]..rec_start[K+1] of rec_idx list the records of tile K's rows:
// its row records in run order, then its column records in band order.
// (BandItem, BandPlan and plan_band live in pb_host.h.)
void launch_pairs_f32_band(hipStream_t s, const float *src, const BandItem *items, int n_items,
                           int n_tiles, const PairParams &pp, int transpose, float *recs);
void launch_band_finish(hipStream_t s, const Geo &geo, const float *recs,
                        const int32_t *rec_start, const int32_t *rec_idx, const double *x,
                        double alpha, double beta, int transpose, double scale1, double scale2,
                        double *y);

// mode / transpose: 0 forward, 1 transposed (x = [l1; l2]).
void launch_pack_sym(hipStream_t s, const Geo &geo, const double *x, float *src, double cx,
                     double cy, double cz, double eps, double sigma, int mode);
void launch_pairs_f32_sym(hipStream_t s, const float *src, const int32_t *items, int n_items,
                          int n_tiles, const PairParams &pp, int transpose, double *rowpart,
                          float *colpart);
void launch_sym_finish(hipStream_t s, const Geo &geo, const double *rowpart,
                       const float *colpart, const int32_t *row_start, int n_tiles,
                       const double *x, double alpha, double beta, int transpose, double scale1,
                       double scale2, double *y);

// Pairwise FP64 sweep on the same work items (forward and transposed).
void launch_pack_sym64(hipStream_t s, const Geo &geo, const double *x, double *src, int mode);
void launch_pairs_f64_sym(hipStream_t s, const double *src, const int32_t *items, int n_items,
                          int n_tiles, const PairParams &pp, int transpose, double *rowpart,
                          double *colpart);
void launch_sym_finish64(hipStream_t s, const Geo &geo, const double *rowpart,
                         const double *colpart, const int32_t *row_start, int n_tiles,
                         const double *x, double alpha, double beta, int transpose, double *y);

// y = diag * x - (1/4pi) [scale1 * sum_c part0; scale2 * sum_c part1]
// (times a_i when transposed)
void launch_matvec_finish(hipStream_t s, const Geo &geo, const double *part, int n_chunks,
                          const double *x, double alpha, double beta, int transpose,
                          double scale1, double scale2, double *y);

// Source terms b = [S1; S2].
void launch_source(hipStream_t s, const Geo &geo, int64_t nc, const double *pos,
                   const double *q, double eps_in, double *b);

// Per-charge reaction potential partials (mode 0) or solid angle (mode 1).
// part[c * ncpad + k]; src is a forward-packed FP64 stream (mode 0).
void launch_charge_pairs(hipStream_t s, const Geo &geo, const double *src, int64_t nc,
                         const double *pos, const Sweep &sw, const PairParams &pp, int mode,
                         double *part, int64_t ncpad);
// per[k] = sum_c part[c][k]; when q and out are given, also
// out[0] = scale * sum_k q_k per[k] (fixed order).
void launch_charge_finish(hipStream_t s, const double *part, int n_chunks, int64_t nc,
                          int64_t ncpad, const double *q, double scale, double *per, double *out);

// Adjoint right-hand side w' = B'^T q (2n).
void launch_adjoint_rhs(hipStream_t s, const Geo &geo, int64_t nc, const double *pos,
                        const double *q, double eps, double kappa, double *w);
// Gradient sweep: fwd = forward-packed xi, adj = transpose-packed lambda';
// part[(o * n_chunks + c) * ncpad + k], o < 8.
void launch_force_pairs(hipStream_t s, const double *fwd, const double *adj, int64_t nc,
                        const double *pos, const Sweep &sw, const PairParams &pp, double *part,
                        int64_t ncpad);
// per [nc] is scratch (receives P'_k); out[0] = E.
void launch_force_finish(hipStream_t s, const double *part, int n_chunks, int64_t nc,
                         int64_t ncpad, const double *q, double half_cu, double inv4pi_eps_in,
                         double *dpos, double *dq, double *per, double *out);

// Leaf blocks of the preconditioner: assemble and invert (one workgroup per
// leaf), and apply y = M^-1 x (trans: M^-T x).  perm lists the collocation
// points leaf by leaf as indices into geo (arrays of stride geo.npad),
// lstart[l]..lstart[l+1] the points of leaf l, boff[l] the offset of its
// (2m)^2 inverse block in inv; pidx/qidx the vector positions of each
// point's phi and psi unknowns.
// pq[e] = perm[e], pq[n + e] = n + perm[e]: the phi and psi slots of the
// elements in leaf order.
void launch_pc_index(hipStream_t s, const int32_t *perm, int64_t n, int64_t *pq);
void launch_pc_build(hipStream_t s, const Geo &geo, const int32_t *perm, const int32_t *lstart,
                     const int64_t *boff, int64_t n_leaves, int max_leaf, double eps,
                     double kappa, double *inv);
void launch_pc_apply(hipStream_t s, const double *inv, const int64_t *boff, const int64_t *pidx,
                     const int64_t *qidx, const int32_t *lstart, int64_t n_leaves,
                     const double *x, int trans, double *y);

// out_k = scale * sum_l q_l / |x_k - y_l| over npts points (skip l == k).
// Counter-calibration probe (pb_probe_valu): PROBE_THREADS threads run chains
// of one operation kind; returns the number of probed operations (summed
// over lanes); each thread writes its result to out[thread].
constexpr int64_t PROBE_THREADS = 1024 * 256;
int64_t launch_probe_valu(hipStream_t s, int kind, double *out);
// ex[k] = exp(-x[k]) and rq[k] = 1/sqrt(y[k]) by the FP64 sweeps' own
// functions, k < n (n < 2^31 * TPB).
void launch_eval_pair_math(hipStream_t s, int64_t n, const double *x, const double *y,
                           double *ex, double *rq);
void launch_point_coulomb(hipStream_t s, int64_t npts, const double *pts, int64_t nc,
                          const double *pos, const double *q, double scale, int skip_self,
                          double *out);
// out[0] = scale * sum_k q_k per[k] (fixed order, one block).
void launch_weighted_total(hipStream_t s, const double *per, const double *q, int64_t nc,
                           double scale, double *out);

// ---- deterministic BLAS-1 on device vectors of length n ----------------
int dot_blocks(int64_t n);
// part[j * nblk + b] = block b's share of <V_j, w> for j < k, and of <w, w> at j = k.
void launch_dots(hipStream_t s, const double *V, int64_t ld, int k, const double *w, int64_t n,
                 double *part, int nblk);
// out[j] = sum_b part[j * nblk + b] in a fixed order, j < ncol.
void launch_reduce_cols(hipStream_t s, const double *part, int nblk, int ncol, double *out);
// w -= sum_{j<k} h[j] V_j
void launch_sub_basis(hipStream_t s, const double *V, int64_t ld, int k, const double *h,
                      double *w, int64_t n);
// v = w / sqrt(*nrm2)   (v = 0 when *nrm2 == 0)
void launch_scale_inv_sqrt(hipStream_t s, const double *w, const double *nrm2, double *v,
                           int64_t n);
// x += sum_{j<k} y[j] V_j
void launch_add_basis(hipStream_t s, const double *V, int64_t ld, int k, const double *y,
                      double *x, int64_t n);
// r = b - ax
void launch_sub(hipStream_t s, const double *b, const double *ax, double *r, int64_t n);
// x += d
void launch_add(hipStream_t s, double *x, const double *d, int64_t n);
void launch_fill(hipStream_t s, double *x, double v, int64_t n);

}  // namespace pbk
