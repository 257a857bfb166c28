// Batched DSBI solves: many independent surfaces of uneven size in shared
// launches.
//
// Layout: the systems' collocation arrays are concatenated, each padded to a
// multiple of PADN, in seven SoA arrays of total length gtot (system b at
// offset goff_b).  Vectors of unknowns use [phi_b (npad_b) | psi_b (npad_b)]
// at offset 2 goff_b, padding entries zero.  Charges are concatenated with
// each system padded to a multiple of TPB.
//
// Pair sweeps run over a work list of equal-sized items (system, target
// block, source tile range), one workgroup per item, longest first, so
// systems from 5,120 to 81,920 triangles share every launch and the
// hardware dispatcher balances the load.
// Each item writes its own partial slot; a second kernel sums a target's
// slots in a fixed order (deterministic, no atomics).
//
// GMRES runs in lockstep over the systems with per-system state on the
// device: Arnoldi (CGS2) reductions are segmented per system, Givens
// rotations, the least-squares update and the convergence tests run in
// one-thread-per-system kernels, and masks switch finished systems off.
// One restart cycle is therefore a fixed kernel sequence: it is captured
// once in a hipGraph and replayed until every system has converged.
// Restart residuals b - A x are always formed with the FP64 sweep; with
// PB_FP32_IR the Arnoldi matvecs use the FP32 sweep, so each cycle is one
// step of iterative refinement.
#include "pb_ctx.h"
#include "pb_device.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <system_error>
#include <thread>
#include <vector>

namespace pbk {

namespace {

using namespace dev;

constexpr int BM_MAX = 32;                    // largest restart length for batches
constexpr int HB = 2 * (BM_MAX + 1) + 2;      // per-system reduction slots
constexpr int H_OFF1 = 0, H_OFF2 = BM_MAX + 1, H_NRM = 2 * (BM_MAX + 1);
constexpr int MV_TILES = 32;                  // source tiles per matvec work item
constexpr int CH_TILES = 16;                  // triangle tiles per charge-sweep item

struct SysDesc {
    int64_t n, npad, goff;      // triangles, padded count, offset in the geometry arrays
    int64_t nc, ncpad, coff;    // charges, padded count, offset in the charge arrays
    int64_t cout;               // offset of the system's charges in caller arrays
    int64_t item0, citem0;      // first matvec / charge-sweep work item
    int32_t nch, cnch;          // chunks per target block / per charge block
    double cx, cy, cz;          // origin for FP32 arithmetic
    int32_t T, rs0;             // pairwise sweeps: tiles, first entry in the row-slot table
    int64_t cp0;                // pairwise sweeps: first tile pair in the column partials
};

struct Item {
    int32_t sys, tb, t0, t1;
};

// Pairwise work item: target tile I of system `sys` against its source tiles
// J0..J1-1; `slot` is its row-partial record.
struct SItem {
    int32_t sys, I, J0, J1, slot, pad0, pad1, pad2;
};


struct GState {
    double H[(BM_MAX + 1) * BM_MAX];
    double cs[BM_MAX], sn[BM_MAX], g[BM_MAX + 1], y[BM_MAX];
    double bnorm, beta, rel, pad_;
    int32_t conv, run, step, k, iters, nres, pad1, pad2;
};

// ---- packing --------------------------------------------------------------

// Charge padding of system b (one block each): entries nc .. ncpad-1 repeat
// the last charge's position with q = 0, so padded charge slots add nothing.
__global__ __launch_bounds__(TPB) void kb_pad_charges(const SysDesc *__restrict__ sd,
                                                      double *__restrict__ pos,
                                                      double *__restrict__ q)
{
    const SysDesc d = sd[blockIdx.x];
    const int64_t last = d.coff + d.nc - 1;
    for (int64_t k = d.nc + threadIdx.x; k < d.ncpad; k += TPB) {
        const int64_t e = d.coff + k;
        pos[3 * e] = pos[3 * last];
        pos[3 * e + 1] = pos[3 * last + 1];
        pos[3 * e + 2] = pos[3 * last + 2];
        q[e] = 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(TPB) void kb_pack(const double *__restrict__ g, int64_t gtot,
                                               const SysDesc *__restrict__ sd,
                                               const int32_t *__restrict__ blk2sys,
                                               const double *__restrict__ x,
                                               Src8<T> *__restrict__ src, int mode, double eps)
{
    const int64_t gi = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const SysDesc d = sd[blk2sys[blockIdx.x]];
    const int64_t j = gi - d.goff;
    const double *xv = x + 2 * d.goff;
    const bool f32 = sizeof(T) == 4;
    const double cx = f32 ? d.cx : 0.0, cy = f32 ? d.cy : 0.0, cz = f32 ? d.cz : 0.0;
    Src8<T> s;
    if (j < d.n) {
        const double a = g[6 * gtot + gi];
        double w, f, pad = 0.0;
        if (mode == 0) {
            w = a * xv[d.npad + j];
            f = a * xv[j];
        } else if (mode == 1) {
            w = xv[j];
            f = xv[d.npad + j];
        } else {
            const double ap = a * xv[d.npad + j];
            w = (1.0 - 1.0 / eps) * ap;
            pad = -ap / eps;
            f = -3.0 * a * xv[j];
        }
        s.x = T(g[gi] - cx);
        s.y = T(g[gtot + gi] - cy);
        s.z = T(g[2 * gtot + gi] - cz);
        s.w = T(w);
        s.mx = T(f * g[3 * gtot + gi]);
        s.my = T(f * g[4 * gtot + gi]);
        s.mz = T(f * g[5 * gtot + gi]);
        s.pad = T(pad);
    } else {
        s.x = T(FAR_SRC - cx);
        s.y = T(0.0);
        s.z = T(0.0);
        s.w = s.mx = s.my = s.mz = s.pad = T(0.0);
    }
    src[gi] = s;
}

// ---- pair sweeps over the work list -----------------------------------------

__global__ __launch_bounds__(TPB) void kb_pairs_f32_fwd(const Src8<float> *__restrict__ src,
                                                        const double *__restrict__ g,
                                                        int64_t gtot,
                                                        const SysDesc *__restrict__ sd,
                                                        const Item *__restrict__ items,
                                                        int64_t n_items,
                                                        const int32_t *__restrict__ mask,
                                                        double eps, double kappa,
                                                        double *__restrict__ part)
{
    __shared__ Src8<float> sh[TILE];
    CoefF32 cf;
    cf.kappa = float(kappa);
    cf.kexp = float(-kappa * 1.4426950408889634074);
    cf.c13 = float((1.0 - 1.0 / eps) / 3.0);
    cf.k23 = float(kappa * kappa / 3.0);
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        if (!mask[w.sys])
            continue;
        const SysDesc d = sd[w.sys];
        const int64_t i = d.goff + (int64_t)w.tb * TPB + threadIdx.x;
        float tg[1][9];
        tg[0][0] = float(g[i] - d.cx);
        tg[0][1] = float(g[gtot + i] - d.cy);
        tg[0][2] = float(g[2 * gtot + i] - d.cz);
        const double nx = g[3 * gtot + i], ny = g[4 * gtot + i], nz = g[5 * gtot + i];
        tg[0][3] = float(nx);
        tg[0][4] = float(ny);
        tg[0][5] = float(nz);
        tg[0][6] = float(-nx / 3.0);
        tg[0][7] = float(-ny / 3.0);
        tg[0][8] = float(-nz / 3.0);
        Acc<float> aP, aQ;
        for (int t = w.t0; t < w.t1; ++t) {
            __syncthreads();
            sh[threadIdx.x] = src[d.goff + (int64_t)t * TILE + threadIdx.x];
            __syncthreads();
            float P[1] = {0.f}, Q[1] = {0.f};
            if (t == w.tb)
                sweep_f32<1, 0, false>(sh, tg, cf, P, Q);
            else
                sweep_f32<1, -1, false>(sh, tg, cf, P, Q);
            aP.add(P[0]);
            aQ.add(Q[0]);
        }
        part[it * TPB + threadIdx.x] = aP.value();
        part[(n_items + it) * TPB + threadIdx.x] = aQ.value();
    }
}

template <typename T, bool TRANS>
__global__ __launch_bounds__(TPB) void kb_pairs(const Src8<T> *__restrict__ src,
                                                const double *__restrict__ g, int64_t gtot,
                                                const SysDesc *__restrict__ sd,
                                                const Item *__restrict__ items, int64_t n_items,
                                                const int32_t *__restrict__ mask, double eps,
                                                double kappa, double *__restrict__ part)
{
    __shared__ Src8<T> sh[TILE];
    PairParams pp;
    pp.eps = eps;
    pp.kappa = kappa;
    pp.cx = pp.cy = pp.cz = 0.0;
    const Coef<T> cf(pp);
    const bool f32 = sizeof(T) == 4;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        if (!mask[w.sys])
            continue;
        const SysDesc d = sd[w.sys];
        const int64_t i = d.goff + (int64_t)w.tb * TPB + threadIdx.x;
        const T xi = T(g[i] - (f32 ? d.cx : 0.0));
        const T yi = T(g[gtot + i] - (f32 ? d.cy : 0.0));
        const T zi = T(g[2 * gtot + i] - (f32 ? d.cz : 0.0));
        const T nxi = T(g[3 * gtot + i]), nyi = T(g[4 * gtot + i]), nzi = T(g[5 * gtot + i]);
        Acc<T> aP, aQ;
        for (int t = w.t0; t < w.t1; ++t) {
            __syncthreads();
            sh[threadIdx.x] = src[d.goff + (int64_t)t * TILE + threadIdx.x];
            __syncthreads();
            T p = T(0), q = T(0);
            if (t == w.tb)
                sweep_tile<T, TRANS, true>(sh, threadIdx.x, xi, yi, zi, nxi, nyi, nzi, cf, p, q);
            else
                sweep_tile<T, TRANS, false>(sh, -1, xi, yi, zi, nxi, nyi, nzi, cf, p, q);
            aP.add(p);
            aQ.add(q);
        }
        const double P = aP.value(), Q = aQ.value();
        part[it * TPB + threadIdx.x] = TRANS ? Q : P;
        part[(n_items + it) * TPB + threadIdx.x] = TRANS ? P : Q;
    }
}

// Preconditioner index tables of the batch: element k of the leaf order is
// point perm[k] = goff + e of system b (sbase[b] <= k < sbase[b + 1]); its
// phi and psi slots in the batch vectors are 2 goff + e and 2 goff + npad + e.
__global__ __launch_bounds__(TPB) void kb_pc_index(const int32_t *__restrict__ perm, int64_t ne,
                                                   const int64_t *__restrict__ sbase,
                                                   const SysDesc *__restrict__ sd, int n_sys,
                                                   int64_t *__restrict__ pidx,
                                                   int64_t *__restrict__ qidx)
{
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k >= ne)
        return;
    int lo = 0, hi = n_sys - 1;   // the system whose range holds k
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (sbase[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    const SysDesc d = sd[lo];
    const int64_t p = (int64_t)perm[k] + d.goff;   // 2 goff + e
    pidx[k] = p;
    qidx[k] = p + d.npad;
}

// ---- pairwise sweeps over the batch ------------------------------------------

// FP32 stream of the pairwise sweep (see k_pack_sym), per system: centred on
// the system's origin and in units of 1/kappa.
__global__ __launch_bounds__(TPB) void kb_pack_sym(const double *__restrict__ g, int64_t gtot,
                                                   const SysDesc *__restrict__ sd,
                                                   const int32_t *__restrict__ blk2sys,
                                                   const double *__restrict__ x,
                                                   Src12 *__restrict__ src, double eps,
                                                   double sigma, int mode)
{
    const int64_t gi = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const SysDesc d = sd[blk2sys[blockIdx.x]];
    const int64_t j = gi - d.goff;
    const double *xv = x + 2 * d.goff;
    Src12 s;
    if (j < d.n) {
        const double a = g[6 * gtot + gi];
        double w1, w2n, nu;
        if (mode) {
            const double w = xv[j] / sigma;
            w1 = (eps - 1.0) * w;
            w2n = eps * w;
            nu = 3.0 * xv[d.npad + j];
        } else {
            const double w = a * xv[d.npad + j] / sigma;
            w1 = (1.0 - 1.0 / eps) * w;
            w2n = -w / eps;
            nu = 3.0 * a * xv[j];
        }
        const double nx = g[3 * gtot + gi], ny = g[4 * gtot + gi], nz = g[5 * gtot + gi];
        s.x = float((g[gi] - d.cx) * sigma);
        s.y = float((g[gtot + gi] - d.cy) * sigma);
        s.z = float((g[2 * gtot + gi] - d.cz) * sigma);
        s.w1 = float(w1);
        s.w2n = float(w2n);
        s.nx = float(-nx);
        s.ny = float(-ny);
        s.nz = float(-nz);
        s.nu = float(nu);
    } else {
        s.x = float((FAR_SRC + 8.0 * double(j - d.n) - d.cx) * sigma);
        s.y = s.z = 0.f;
        s.w1 = s.w2n = s.nu = 0.f;
        s.nx = s.ny = s.nz = 0.f;
    }
    s.res0 = s.res1 = s.res2 = 0.f;
    src[gi] = s;
}

// FP64 stream of the pairwise sweep (see k_pack_sym64), mode 0 forward, 1 transposed.
__global__ __launch_bounds__(TPB) void kb_pack_sym64(const double *__restrict__ g, int64_t gtot,
                                                     const SysDesc *__restrict__ sd,
                                                     const int32_t *__restrict__ blk2sys,
                                                     const double *__restrict__ x,
                                                     Src8d *__restrict__ src, int mode)
{
    const int64_t gi = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const SysDesc d = sd[blk2sys[blockIdx.x]];
    const int64_t j = gi - d.goff;
    const double *xv = x + 2 * d.goff;
    Src8d s;
    if (j < d.n) {
        const double a = g[6 * gtot + gi];
        const double w = mode ? xv[j] : a * xv[d.npad + j];
        const double f = mode ? xv[d.npad + j] : a * xv[j];
        s.x = g[gi];
        s.y = g[gtot + gi];
        s.z = g[2 * gtot + gi];
        s.w = w;
        s.nx = g[3 * gtot + gi];
        s.ny = g[4 * gtot + gi];
        s.nz = g[5 * gtot + gi];
        s.f = f;
    } else {
        s.x = FAR_SRC + 8.0 * double(j - d.n);
        s.y = s.z = 0.0;
        s.w = s.f = s.nx = s.ny = s.nz = 0.0;
    }
    src[gi] = s;
}

template <bool SCALED>
__global__ __launch_bounds__(SYM_NT, SYM_MIN_WAVES) void kb_pairs_f32_sym(const Src12 *__restrict__ src,
                                                        const SysDesc *__restrict__ sd,
                                                        const SItem *__restrict__ items,
                                                        int64_t n_items,
                                                        const int32_t *__restrict__ mask,
                                                        double eps, double kappa,
                                                        double *__restrict__ rowpart,
                                                        float *__restrict__ colpart)
{
    __shared__ SrcTileF32 sh;
    __shared__ float colw[SYM_NT / 64][2 * TILE];
    const CoefF32 cf = coef_f32(eps, kappa, SCALED);
    for (int64_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        const SItem w = items[k];
        if (!mask[w.sys])
            continue;
        const SysDesc d = sd[w.sys];
        sym_item_f32<SCALED>(src + d.goff, w.I, w.J0, w.J1, d.T, cf,
                             rowpart + (int64_t)w.slot * (2 * TILE),
                             colpart + d.cp0 * (2 * TILE), sh, colw);
    }
}

template <bool TRANS>
__global__ __launch_bounds__(SYM64_NT, SYM64_MIN_WAVES) void kb_pairs_f64_sym(const Src8d *__restrict__ src,
                                                        const SysDesc *__restrict__ sd,
                                                        const SItem *__restrict__ items,
                                                        int64_t n_items,
                                                        const int32_t *__restrict__ mask,
                                                        double eps, double kappa,
                                                        double *__restrict__ rowpart,
                                                        double *__restrict__ colpart)
{
    __shared__ Src8d sh[SYM64_NS];
    __shared__ double colw[SYM64_NT / 64][2 * SYM64_NS];
    __shared__ double acc[2 * SYM64_TT][SYM64_NT];
    PairParams pp;
    pp.eps = eps;
    pp.kappa = kappa;
    pp.cx = pp.cy = pp.cz = 0.0;
    const Coef<double> cf(pp);
    for (int64_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        const SItem w = items[k];
        if (!mask[w.sys])
            continue;
        const SysDesc d = sd[w.sys];
        sym_item_f64<TRANS>(src + d.goff, w.I, w.J0, w.J1, d.T, cf,
                            rowpart + (int64_t)w.slot * (2 * TILE),
                            colpart + d.cp0 * (2 * TILE), sh, colw, acc);
    }
}

// Rows of masked systems from the pairwise partials: the item rows of the
// point's tile, then the contributions of every lower tile, in that order.
template <typename CT>
__global__ __launch_bounds__(TPB) void kb_sym_finish(const double *__restrict__ rowpart,
                                                     const CT *__restrict__ colpart,
                                                     const int32_t *__restrict__ rs,
                                                     const double *__restrict__ g, int64_t gtot,
                                                     const SysDesc *__restrict__ sd,
                                                     const int32_t *__restrict__ blk2sys,
                                                     const int32_t *__restrict__ mask,
                                                     const double *__restrict__ x, double alpha,
                                                     double beta, int trans, double scale1,
                                                     double scale2, double *__restrict__ y)
{
    const int b = blk2sys[blockIdx.x];
    if (!mask[b])
        return;
    const SysDesc d = sd[b];
    const int64_t gi = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t j = gi - d.goff;
    const double *xv = x + 2 * d.goff;
    double *yv = y + 2 * d.goff;
    if (j >= d.n) {
        yv[j] = 0.0;
        yv[d.npad + j] = 0.0;
        return;
    }
    const int K = (int)(j / TILE), l = (int)(j % TILE);
    double s1 = 0.0, s2 = 0.0;
    for (int q = rs[d.rs0 + K]; q < rs[d.rs0 + K + 1]; ++q) {
        s1 += rowpart[(int64_t)q * (2 * TILE) + l];
        s2 += rowpart[(int64_t)q * (2 * TILE) + TILE + l];
    }
    for (int I = 0; I < K; ++I) {
        const CT *cp = colpart + (d.cp0 + sym_pair_index(I, K, d.T)) * (2 * TILE);
        s1 += (double)cp[l];
        s2 += (double)cp[TILE + l];
    }
    if (trans) {
        const double sc = g[6 * gtot + gi] * INV_4PI;
        yv[j] = alpha * xv[j] - sc * scale2 * s2;
        yv[d.npad + j] = beta * xv[d.npad + j] - sc * scale1 * s1;
    } else {
        yv[j] = alpha * xv[j] - INV_4PI * scale1 * s1;
        yv[d.npad + j] = beta * xv[d.npad + j] - INV_4PI * scale2 * s2;
    }
}

// y = diag x - (1/4pi) [scale1 * row1 sums; row2 sums] for masked systems.
__global__ __launch_bounds__(TPB) void kb_finish(const double *__restrict__ part, int64_t n_items,
                                                 const double *__restrict__ g, int64_t gtot,
                                                 const SysDesc *__restrict__ sd,
                                                 const int32_t *__restrict__ blk2sys,
                                                 const int32_t *__restrict__ mask,
                                                 const double *__restrict__ x, double alpha,
                                                 double beta, int trans, double scale1,
                                                 double *__restrict__ y)
{
    const int b = blk2sys[blockIdx.x];
    if (!mask[b])
        return;
    const SysDesc d = sd[b];
    const int64_t gi = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t j = gi - d.goff;
    const double *xv = x + 2 * d.goff;
    double *yv = y + 2 * d.goff;
    if (j >= d.n) {
        yv[j] = 0.0;
        yv[d.npad + j] = 0.0;
        return;
    }
    const int64_t tb = j / TPB;
    const int64_t s0 = d.item0 + tb * d.nch;
    double s1 = 0.0, s2 = 0.0;
    for (int c = 0; c < d.nch; ++c) {
        s1 += part[(s0 + c) * TPB + threadIdx.x];
        s2 += part[(n_items + s0 + c) * TPB + threadIdx.x];
    }
    const double sc = trans ? g[6 * gtot + gi] * INV_4PI : INV_4PI;
    yv[j] = alpha * xv[j] - sc * scale1 * s1;
    yv[d.npad + j] = beta * xv[d.npad + j] - sc * s2;
}

// ---- sources and the adjoint right-hand side --------------------------------

__global__ __launch_bounds__(TPB) void kb_source(const double *__restrict__ g, int64_t gtot,
                                                 const SysDesc *__restrict__ sd,
                                                 const int32_t *__restrict__ blk2sys,
                                                 const double *__restrict__ pos,
                                                 const double *__restrict__ q, double scale,
                                                 int adjoint, double eps, double kappa,
                                                 double *__restrict__ out)
{
    __shared__ double4 sh[TILE];
    const SysDesc d = sd[blk2sys[blockIdx.x]];
    const int64_t gi = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t j = gi - d.goff;
    const double xi = g[gi], yi = g[gtot + gi], zi = g[2 * gtot + gi];
    const double nxi = g[3 * gtot + gi], nyi = g[4 * gtot + gi], nzi = g[5 * gtot + gi];
    const double epsm1 = eps - 1.0;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t t0 = 0; t0 < d.nc; t0 += TILE) {
        __syncthreads();
        const int64_t k = t0 + threadIdx.x;
        const int64_t kg = d.coff + k;
        sh[threadIdx.x] = (k < d.nc)
                              ? make_double4(pos[3 * kg], pos[3 * kg + 1], pos[3 * kg + 2], q[kg])
                              : make_double4(FAR_SRC, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = (int)min((int64_t)TILE, d.nc - t0);
        for (int kk = 0; kk < cnt; ++kk) {
            const double4 c = sh[kk];
            const double dx = xi - c.x, dy = yi - c.y, dz = zi - c.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsqrt_t(r2);
            const double cxd = nxi * dx + nyi * dy + nzi * dz;
            if (!adjoint) {
                s1 += c.w * ir;
                s2 += c.w * cxd * (ir * ir * ir);
            } else {
                const double kr = kappa * (r2 * ir);
                const double e = exp_neg(kr);
                const double em1 = e - 1.0;
                const double g2 = fma(eps, fma(kr, e, em1), epsm1);
                s1 = fma(c.w * g2 * cxd, ir * ir * ir, s1);
                s2 = fma(c.w * em1, ir, s2);
            }
        }
    }
    double *ov = out + 2 * d.goff;
    if (j < d.n) {
        if (!adjoint) {
            ov[j] = s1 * scale;
            ov[d.npad + j] = -s2 * scale;
        } else {
            const double a = g[6 * gtot + gi];
            ov[j] = -a * s1;
            ov[d.npad + j] = -a * s2;
        }
    } else {
        ov[j] = 0.0;
        ov[d.npad + j] = 0.0;
    }
}

// ---- charge-target sweeps ----------------------------------------------------
// MODE 0: reaction potential P'_k; MODE 1: solid angle; MODE 2: the eight
// gradient sums of the single-system force sweep (fwd and adj streams).
template <int MODE>
__global__ __launch_bounds__(TPB) void kb_charge_pairs(const Src8<double> *__restrict__ fwd,
                                                       const Src8<double> *__restrict__ adj,
                                                       const SysDesc *__restrict__ sd,
                                                       const Item *__restrict__ items,
                                                       int64_t n_items,
                                                       const double *__restrict__ pos,
                                                       double eps, double kappa,
                                                       double *__restrict__ part)
{
    constexpr int K = MODE == 2 ? 8 : 1;
    __shared__ Src8<double> shf[TILE];
    __shared__ Src8<double> sha[MODE == 2 ? TILE : 1];
    const double epsm1 = eps - 1.0, ek2 = eps * kappa * kappa;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SysDesc d = sd[w.sys];
        int64_t k = (int64_t)w.tb * TPB + threadIdx.x;
        if (k >= d.nc)
            k = d.nc - 1;
        const int64_t kg = d.coff + k;
        const double yx = pos[3 * kg], yy = pos[3 * kg + 1], yz = pos[3 * kg + 2];
        double acc[K];
#pragma unroll
        for (int o = 0; o < K; ++o)
            acc[o] = 0.0;
        for (int t = w.t0; t < w.t1; ++t) {
            __syncthreads();
            shf[threadIdx.x] = fwd[d.goff + (int64_t)t * TILE + threadIdx.x];
            if (MODE == 2)
                sha[threadIdx.x] = adj[d.goff + (int64_t)t * TILE + threadIdx.x];
            __syncthreads();
            for (int jj = 0; jj < TILE; ++jj) {
                const Src8<double> f = shf[jj];
                const double dx = yx - f.x, dy = yy - f.y, dz = yz - f.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double ir = rsqrt_t(r2);
                const double ir2 = ir * ir;
                const double u = ir2 * ir;
                const double md = f.mx * dx + f.my * dy + f.mz * dz;
                if (MODE == 1) {
                    acc[0] = fma(-md, u, acc[0]);
                    continue;
                }
                const double kr = kappa * (r2 * ir);
                const double e = exp_neg(kr);
                const double em1 = e - 1.0;
                const double tm1 = fma(kr, e, em1);
                const double g2 = fma(eps, tm1, epsm1);
                acc[0] = fma(-em1, ir * f.w, acc[0]);
                acc[0] = fma(g2 * md, u, acc[0]);
                if (MODE == 2) {
                    const Src8<double> a = sha[jj];
                    const double cd = f.w * tm1 - ek2 * e * md - 3.0 * g2 * md * ir2;
                    acc[1] = fma(u, fma(dx, cd, g2 * f.mx), acc[1]);
                    acc[2] = fma(u, fma(dy, cd, g2 * f.my), acc[2]);
                    acc[3] = fma(u, fma(dz, cd, g2 * f.mz), acc[3]);
                    const double pd = a.mx * dx + a.my * dy + a.mz * dz;
                    acc[4] = fma(a.w, ir, acc[4]);
                    acc[4] = fma(pd, u, acc[4]);
                    const double ca = a.w + 3.0 * pd * ir2;
                    acc[5] = fma(u, fma(-dx, ca, a.mx), acc[5]);
                    acc[6] = fma(u, fma(-dy, ca, a.my), acc[6]);
                    acc[7] = fma(u, fma(-dz, ca, a.mz), acc[7]);
                }
            }
        }
#pragma unroll
        for (int o = 0; o < K; ++o)
            part[((int64_t)o * n_items + it) * TPB + threadIdx.x] = acc[o];
    }
}

// Per-charge sums over a charge block's chunks (grid over all charge blocks).
template <int K>
__global__ __launch_bounds__(TPB) void kb_charge_sum(const double *__restrict__ part,
                                                     int64_t n_items,
                                                     const SysDesc *__restrict__ sd,
                                                     const int32_t *__restrict__ cblk2sys,
                                                     double *__restrict__ per)
{
    const int b = cblk2sys[blockIdx.x];
    const SysDesc d = sd[b];
    const int64_t kg = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t k = kg - d.coff;
    if (k >= d.nc)
        return;
    const int64_t cb = k / TPB;
    const int64_t s0 = d.citem0 + cb * d.cnch;
#pragma unroll
    for (int o = 0; o < K; ++o) {
        double s = 0.0;
        for (int c = 0; c < d.cnch; ++c)
            s += part[((int64_t)o * n_items + s0 + c) * TPB + threadIdx.x];
        per[kg * K + o] = s;
    }
}

// E_b = scale * sum_k q_k per[k K] over system b's charges (one block per system).
__global__ __launch_bounds__(TPB) void kb_energy(const double *__restrict__ per, int K,
                                                 const double *__restrict__ q,
                                                 const SysDesc *__restrict__ sd, double scale,
                                                 double *__restrict__ e)
{
    __shared__ double sh[TPB / 64];
    const SysDesc d = sd[blockIdx.x];
    double tot = 0.0;
    for (int64_t k = threadIdx.x; k < d.nc; k += TPB)
        tot += q[d.coff + k] * per[(d.coff + k) * K];
    const double r = block_sum(tot, sh);
    if (threadIdx.x == 0)
        e[blockIdx.x] = scale * r;
}

// Gradients in caller layout from the eight per-charge sums.
__global__ __launch_bounds__(TPB) void kb_force_out(const double *__restrict__ per,
                                                    const double *__restrict__ q,
                                                    const SysDesc *__restrict__ sd,
                                                    const int32_t *__restrict__ cblk2sys,
                                                    double half_cu, double inv4pi_eps_in,
                                                    double *__restrict__ dpos,
                                                    double *__restrict__ dq)
{
    const SysDesc d = sd[cblk2sys[blockIdx.x]];
    const int64_t kg = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t k = kg - d.coff;
    if (k >= d.nc)
        return;
    const double *v = per + kg * 8;
    const int64_t o = d.cout + k;
    dq[o] = half_cu * (v[0] + inv4pi_eps_in * v[4]);
    for (int c = 0; c < 3; ++c)
        dpos[3 * o + c] = half_cu * q[kg] * (v[1 + c] + inv4pi_eps_in * v[5 + c]);
}

// ---- segmented BLAS-1 (vector blocks never straddle systems) ----------------

__global__ __launch_bounds__(TPB) void kb_dots(const double *__restrict__ V, int64_t ld, int k,
                                               const double *__restrict__ w,
                                               double *__restrict__ part, int64_t nvb)
{
    __shared__ double sh[TPB / 64];
    const int j = blockIdx.y;
    const double *a = (j < k) ? V + (int64_t)j * ld : w;
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const double r = block_sum(a[i] * w[i], sh);
    if (threadIdx.x == 0)
        part[(int64_t)j * nvb + blockIdx.x] = r;
}

// red[b * HB + off + j] = sum of system b's block partials of column j.
__global__ __launch_bounds__(TPB) void kb_red(const double *__restrict__ part, int64_t nvb,
                                              const SysDesc *__restrict__ sd, int off,
                                              double *__restrict__ red)
{
    __shared__ double sh[TPB / 64];
    const int b = blockIdx.x, j = blockIdx.y;
    const SysDesc d = sd[b];
    const int64_t v0 = 2 * d.goff / TPB, nb = 2 * d.npad / TPB;
    double s = 0.0;
    for (int64_t v = threadIdx.x; v < nb; v += TPB)
        s += part[(int64_t)j * nvb + v0 + v];
    const double r = block_sum(s, sh);
    if (threadIdx.x == 0)
        red[(int64_t)b * HB + off + j] = r;
}

__global__ __launch_bounds__(TPB) void kb_sub_basis(const double *__restrict__ V, int64_t ld,
                                                    int k, const double *__restrict__ red,
                                                    int off, const int32_t *__restrict__ vblk2sys,
                                                    double *__restrict__ w)
{
    const int b = vblk2sys[blockIdx.x];
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    double s = w[i];
    for (int j = 0; j < k; ++j)
        s -= red[(int64_t)b * HB + off + j] * V[(int64_t)j * ld + i];
    w[i] = s;
}

__global__ __launch_bounds__(TPB) void kb_scale(const double *__restrict__ w,
                                                const double *__restrict__ red,
                                                const int32_t *__restrict__ vblk2sys,
                                                double *__restrict__ v)
{
    const int b = vblk2sys[blockIdx.x];
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const double s2 = red[(int64_t)b * HB + H_NRM];
    v[i] = (s2 > 0.0) ? w[i] / sqrt(s2) : 0.0;
}

__global__ __launch_bounds__(TPB) void kb_add_basis(const double *__restrict__ V, int64_t ld,
                                                    int m, const GState *__restrict__ st,
                                                    const int32_t *__restrict__ vblk2sys,
                                                    double *__restrict__ x)
{
    const int b = vblk2sys[blockIdx.x];
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const GState &s = st[b];
    if (!s.run)
        return;
    double acc = 0.0;
    for (int j = 0; j < s.k && j < m; ++j)
        acc += s.y[j] * V[(int64_t)j * ld + i];
    x[i] += acc;
}

__global__ __launch_bounds__(TPB) void kb_axpby(const double *__restrict__ a,
                                                const double *__restrict__ b, double beta,
                                                double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    out[i] = a[i] + beta * b[i];
}

__global__ __launch_bounds__(TPB) void kb_fill(double *__restrict__ x, double v)
{
    x[(int64_t)blockIdx.x * TPB + threadIdx.x] = v;
}

// ---- per-system GMRES control (one thread per system) ------------------------

__global__ void kb_init(GState *__restrict__ st, const double *__restrict__ red, int n_sys)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_sys)
        return;
    GState &s = st[b];
    s.bnorm = sqrt(red[(int64_t)b * HB + H_NRM]);
    s.beta = s.bnorm;
    s.rel = 1.0;
    s.conv = (s.bnorm == 0.0);
    s.run = 0;
    s.step = 0;
    s.k = 0;
    s.iters = 0;
    s.nres = 0;
}

// Start of a restart cycle: true residual norm -> convergence test -> masks.
// Only systems that ran the cycle just finished (or all of them at the first
// start) have a fresh residual in red; the others keep their state.
__global__ void kb_begin(GState *__restrict__ st, const double *__restrict__ red, int n_sys,
                         int m, double tol, int max_iter, int first,
                         int32_t *__restrict__ mask_step, int32_t *__restrict__ mask_run,
                         int32_t *__restrict__ active)
{
    __shared__ double sh[4];
    double cnt = 0.0;
    for (int b = threadIdx.x; b < n_sys; b += blockDim.x) {
        GState &s = st[b];
        const int fresh = first || s.run;
        if (s.run)
            s.nres += 1;   // the residual just formed used one matvec
        if (fresh && !s.conv) {
            s.beta = sqrt(red[(int64_t)b * HB + H_NRM]);
            s.rel = s.bnorm > 0.0 ? s.beta / s.bnorm : 0.0;
            if (s.rel <= tol)
                s.conv = 1;
        }
        const int go = fresh && !s.conv && s.iters < max_iter && isfinite(s.beta);
        s.run = go;
        s.step = go;
        s.k = 0;
        for (int i = 0; i <= m; ++i)
            s.g[i] = 0.0;
        for (int i = 0; i < m; ++i)
            s.y[i] = 0.0;
        s.g[0] = s.beta;
        mask_step[b] = go;
        mask_run[b] = go;
        cnt += go;
    }
    const double tot = block_sum(cnt, sh);
    if (threadIdx.x == 0)
        active[0] = (int32_t)tot;
}

// Arnoldi step j of each running system: Hessenberg column, Givens rotations,
// and the end of the cycle's Krylov steps.  An FP64 cycle steps until its
// residual estimate reaches tol |b|.  An FP32 cycle is one refinement step:
// as the single-system inner solves, it steps until the estimate reaches
// max(inner |r|, 0.3 tol |b|) (at most |r| / 2; inner > 0), |r| the cycle's
// starting residual, so that the FP64 residual formed after it lands below
// tol rather than at it.
__global__ void kb_givens(GState *__restrict__ st, const double *__restrict__ red, int n_sys,
                          int j, int m, double tol, double inner, int max_iter,
                          int32_t *__restrict__ mask_step)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_sys)
        return;
    GState &s = st[b];
    if (!s.step)
        return;
    const double *h = red + (int64_t)b * HB;
    double *H = s.H;
    for (int i = 0; i <= j; ++i)
        H[i * m + j] = h[H_OFF1 + i] + h[H_OFF2 + i];
    const double hn = sqrt(h[H_NRM]);
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = s.cs[i] * H[i * m + j] + s.sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -s.sn[i] * H[i * m + j] + s.cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
    }
    const double den = hypot(H[j * m + j], H[(j + 1) * m + j]);
    s.cs[j] = H[j * m + j] / den;
    s.sn[j] = H[(j + 1) * m + j] / den;
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    s.g[j + 1] = -s.sn[j] * s.g[j];
    s.g[j] = s.cs[j] * s.g[j];
    s.k = j + 1;
    s.iters += 1;
    const double target = inner > 0.0
                              ? fmin(0.5 * s.beta, fmax(inner * s.beta, 0.3 * tol * s.bnorm))
                              : tol * s.bnorm;
    if (fabs(s.g[j + 1]) <= target || s.iters >= max_iter || !(hn > 0.0) || !isfinite(hn)) {
        s.step = 0;
        mask_step[b] = 0;
    }
}

// Least-squares solution y of the cycle (back substitution).
__global__ void kb_solve_y(GState *__restrict__ st, int n_sys, int m)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_sys)
        return;
    GState &s = st[b];
    if (!s.run)
        return;
    for (int i = s.k - 1; i >= 0; --i) {
        double v = s.g[i];
        for (int l = i + 1; l < s.k; ++l)
            v -= s.H[i * m + l] * s.y[l];
        s.y[i] = v / s.H[i * m + i];
    }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

// ======================= host driver ============================================

namespace {

struct BatchPlan {
    int n_sys = 0;
    int64_t gtot = 0, ctot = 0;
    std::vector<SysDesc> sd;
    std::vector<Item> items, citems;
    std::vector<int32_t> blk2sys, vblk2sys, cblk2sys;
    // pairwise sweeps: work items (longest first), row-slot table, tile pairs
    std::vector<SItem> sitems;
    std::vector<int32_t> rs;
    int64_t n_slots = 0, cptot = 0;
    double sigma_min = 1.0;   // FP32 length unit bound: 1 / the largest system's length scale
};

// Pairwise work items: row tile I of every system against its tiles I.. in
// runs of `tiles` source tiles, longest first; rebuilt when the autotuner
// tries another run length (the tile-pair records do not depend on it).
void plan_sym_items(BatchPlan &P, int tiles)
{
    P.sitems.clear();
    P.rs.clear();
    P.n_slots = 0;
    for (int b = 0; b < P.n_sys; ++b) {
        SysDesc &d = P.sd[b];
        const int nt = d.T;
        d.rs0 = (int32_t)P.rs.size();
        for (int I = 0; I < nt; ++I) {
            P.rs.push_back((int32_t)P.n_slots);
            for (int J0 = I; J0 < nt; J0 += tiles) {
                P.sitems.push_back({b, I, J0, std::min(nt, J0 + tiles), (int32_t)P.n_slots, 0,
                                    0, 0});
                ++P.n_slots;
            }
        }
        P.rs.push_back((int32_t)P.n_slots);
    }
    std::stable_sort(P.sitems.begin(), P.sitems.end(), [](const SItem &a, const SItem &b) {
        return a.J1 - a.J0 > b.J1 - b.J0;
    });
}

void plan_batch(BatchPlan &P, int n_sys, const pb_surface *surf, const pb_charges *chg,
                int sym_tiles)
{
    P.n_sys = n_sys;
    P.sd.resize(n_sys);
    int64_t goff = 0, coff = 0, cout = 0;
    for (int b = 0; b < n_sys; ++b) {
        SysDesc &d = P.sd[b];
        d.n = surf[b].n_tri;
        d.npad = round_up(d.n, PADN);
        d.goff = goff;
        goff += d.npad;
        d.nc = chg[b].n;
        d.ncpad = round_up(d.nc, TPB);
        d.coff = coff;
        coff += d.ncpad;
        d.cout = cout;
        cout += d.nc;
        d.cx = d.cy = d.cz = 0.0;
    }
    P.gtot = goff;
    P.ctot = coff;
    for (int b = 0; b < n_sys; ++b) {
        SysDesc &d = P.sd[b];
        const int ntb = (int)(d.npad / TPB), nt = (int)(d.npad / TILE);
        d.nch = (nt + MV_TILES - 1) / MV_TILES;
        d.item0 = (int64_t)P.items.size();
        for (int tb = 0; tb < ntb; ++tb)
            for (int c = 0; c < d.nch; ++c)
                P.items.push_back({b, tb, c * MV_TILES, std::min(nt, (c + 1) * MV_TILES)});
        const int ncb = (int)(d.ncpad / TPB);
        d.cnch = (nt + CH_TILES - 1) / CH_TILES;
        d.citem0 = (int64_t)P.citems.size();
        for (int cb = 0; cb < ncb; ++cb)
            for (int c = 0; c < d.cnch; ++c)
                P.citems.push_back({b, cb, c * CH_TILES, std::min(nt, (c + 1) * CH_TILES)});
        for (int64_t k = 0; k < d.npad / TPB; ++k)
            P.blk2sys.push_back(b);
        for (int64_t k = 0; k < 2 * d.npad / TPB; ++k)
            P.vblk2sys.push_back(b);
        for (int64_t k = 0; k < d.ncpad / TPB; ++k)
            P.cblk2sys.push_back(b);
        // pairwise sweeps: T tiles, row-slot table at rs0, tile pairs at cp0
        d.T = nt;
        d.cp0 = P.cptot;
        P.cptot += (int64_t)nt * (nt - 1) / 2;
    }
    plan_sym_items(P, sym_tiles);
}

struct BatchDev {
    double *g = nullptr;            // 7 * gtot
    SysDesc *sd = nullptr;
    Item *items = nullptr, *citems = nullptr;
    int32_t *blk2sys = nullptr, *vblk2sys = nullptr, *cblk2sys = nullptr;
    int32_t *mask_step = nullptr, *mask_run = nullptr, *active = nullptr;
    double *pos = nullptr, *q = nullptr;
    void *src = nullptr;            // 16 doubles per collocation point
    double *part = nullptr;
    SItem *sitems = nullptr;         // pairwise sweeps
    int32_t *rs = nullptr;
    double *srow = nullptr;
    void *scol = nullptr;            // FP32 or FP64 column partials
    double *x = nullptr, *b = nullptr, *w = nullptr, *r = nullptr, *t = nullptr, *lam = nullptr;
    double *pw = nullptr, *pb = nullptr;
    double *V = nullptr;
    // block-diagonal leaf preconditioner over all systems (0 leaves: off)
    int64_t pc_leaves = 0;
    int32_t *pc_perm = nullptr, *pc_start = nullptr;
    int64_t *pc_boff = nullptr, *pc_pidx = nullptr, *pc_qidx = nullptr;
    double *pc_inv = nullptr;
    GState *st = nullptr;
    double *red = nullptr, *dpart = nullptr, *per = nullptr, *e = nullptr;
    int64_t vtot = 0, nvb = 0, ld = 0;
};

// One workgroup per work item (the kernels also accept fewer and stride).
inline unsigned item_grid(int64_t n_items)
{
    return (unsigned)std::min<int64_t>(n_items, INT32_MAX);
}

void pc_apply_batch(hipStream_t s, const BatchDev &D, int trans, const double *x, double *y)
{
    launch_pc_apply(s, D.pc_inv, D.pc_boff, D.pc_pidx, D.pc_qidx, D.pc_start, D.pc_leaves, x,
                    trans, y);
}

// y = A x (or A^T x) for the systems in `mask`, with the sweep kind the
// context selects: pairwise (default) or per target.
void enqueue_matvec(pb_ctx *c, const BatchPlan &P, BatchDev &D, bool f32, int trans,
                    const int32_t *mask, double eps, double kap, const double *x, double *y)
{
    hipStream_t s = c->stream;
    const int64_t ni = (int64_t)P.items.size();
    const unsigned grid = item_grid(ni);
    const unsigned gb = nblk(P.gtot);
    const double alpha = 0.5 * (1.0 + eps), beta = 0.5 * (1.0 + 1.0 / eps);
    const int64_t nsi = (int64_t)P.sitems.size();
    if (f32 && c->f32_tpt == PB_SWEEP_PAIRWISE) {
        // transposed: stream mode 1, eps -> 1/eps in the pair constant, rows
        // swapped and scaled by -sigma^2/eps and sigma^3 (as in the single-
        // system sweep)
        const unsigned sgrid = item_grid(nsi);
        const double sig = f32_sigma(kap, P.sigma_min);
        const double keps = trans ? 1.0 / eps : eps;
        hipLaunchKernelGGL(kb_pack_sym, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd, D.blk2sys,
                           x, reinterpret_cast<Src12 *>(D.src), eps, sig, trans ? 1 : 0);
        if (kap > 0.0 && sig == kap)
            hipLaunchKernelGGL(kb_pairs_f32_sym<true>, dim3(sgrid), dim3(SYM_NT), 0, s,
                               reinterpret_cast<const Src12 *>(D.src), D.sd, D.sitems, nsi, mask,
                               keps, 1.0, D.srow, static_cast<float *>(D.scol));
        else
            hipLaunchKernelGGL(kb_pairs_f32_sym<false>, dim3(sgrid), dim3(SYM_NT), 0, s,
                               reinterpret_cast<const Src12 *>(D.src), D.sd, D.sitems, nsi, mask,
                               keps, kap / sig, D.srow, static_cast<float *>(D.scol));
        const double s1 = trans ? -sig * sig / eps : eps * sig * sig;
        hipLaunchKernelGGL(kb_sym_finish<float>, dim3(gb), dim3(TPB), 0, s, D.srow,
                           static_cast<const float *>(D.scol), D.rs, D.g, P.gtot, D.sd,
                           D.blk2sys, mask, x, alpha, beta, trans ? 1 : 0, s1, sig * sig * sig,
                           y);
        return;
    }
    if (!f32 && c->f64_kind == PB_SWEEP_PAIRWISE) {
        const unsigned sgrid = item_grid(nsi);
        hipLaunchKernelGGL(kb_pack_sym64, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, x, reinterpret_cast<Src8d *>(D.src), trans ? 1 : 0);
        if (trans)
            hipLaunchKernelGGL(kb_pairs_f64_sym<true>, dim3(sgrid), dim3(SYM64_NT), 0, s,
                               reinterpret_cast<const Src8d *>(D.src), D.sd, D.sitems, nsi, mask,
                               eps, kap, D.srow, static_cast<double *>(D.scol));
        else
            hipLaunchKernelGGL(kb_pairs_f64_sym<false>, dim3(sgrid), dim3(SYM64_NT), 0, s,
                               reinterpret_cast<const Src8d *>(D.src), D.sd, D.sitems, nsi, mask,
                               eps, kap, D.srow, static_cast<double *>(D.scol));
        hipLaunchKernelGGL(kb_sym_finish<double>, dim3(gb), dim3(TPB), 0, s, D.srow,
                           static_cast<const double *>(D.scol), D.rs, D.g, P.gtot, D.sd,
                           D.blk2sys, mask, x, alpha, beta, trans, 1.0, 1.0, y);
        return;
    }
    if (f32 && !trans) {
        hipLaunchKernelGGL(kb_pack<float>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, x, reinterpret_cast<Src8<float> *>(D.src), 2, eps);
        hipLaunchKernelGGL(kb_pairs_f32_fwd, dim3(grid), dim3(TPB), 0, s,
                           reinterpret_cast<const Src8<float> *>(D.src), D.g, P.gtot, D.sd,
                           D.items, ni, mask, eps, kap, D.part);
    } else if (f32) {
        hipLaunchKernelGGL(kb_pack<float>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, x, reinterpret_cast<Src8<float> *>(D.src), 1, eps);
        hipLaunchKernelGGL((kb_pairs<float, true>), dim3(grid), dim3(TPB), 0, s,
                           reinterpret_cast<const Src8<float> *>(D.src), D.g, P.gtot, D.sd,
                           D.items, ni, mask, eps, kap, D.part);
    } else {
        hipLaunchKernelGGL(kb_pack<double>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, x, reinterpret_cast<Src8<double> *>(D.src), trans ? 1 : 0,
                           eps);
        if (trans)
            hipLaunchKernelGGL((kb_pairs<double, true>), dim3(grid), dim3(TPB), 0, s,
                               reinterpret_cast<const Src8<double> *>(D.src), D.g, P.gtot, D.sd,
                               D.items, ni, mask, eps, kap, D.part);
        else
            hipLaunchKernelGGL((kb_pairs<double, false>), dim3(grid), dim3(TPB), 0, s,
                               reinterpret_cast<const Src8<double> *>(D.src), D.g, P.gtot, D.sd,
                               D.items, ni, mask, eps, kap, D.part);
    }
    hipLaunchKernelGGL(kb_finish, dim3(gb), dim3(TPB), 0, s, D.part, ni, D.g, P.gtot, D.sd,
                       D.blk2sys, mask, x, alpha, beta, trans, (f32 && !trans) ? eps : 1.0, y);
}

// One restart cycle (m Arnoldi steps, update, FP64 residual, next start) on
// the stream; captured into a graph by the caller.  With the preconditioner
// the Krylov space is that of M^-1 A and residuals are M^-1 (rhs - A x).
int enqueue_cycle(pb_ctx *c, const BatchPlan &P, BatchDev &D, const pb_params *p, int trans,
                  const double *rhs, double *x)
{
    hipStream_t s = c->stream;
    const int m = p->restart, ns = P.n_sys;
    const double eps = p->eps_out / p->eps_in, kap = p->kappa;
    const unsigned vb = (unsigned)D.nvb;
    const unsigned sb = (unsigned)((ns + 255) / 256);
    const bool f32 = p->precision == PB_FP32_IR;
    for (int j = 0; j < m; ++j) {
        const double *vj = D.V + (int64_t)j * D.ld;
        enqueue_matvec(c, P, D, f32, trans, D.mask_step, eps, kap, vj, D.w);
        double *wv = D.w;
        if (D.pc_leaves > 0) {
            pc_apply_batch(s, D, trans, D.w, D.pw);
            wv = D.pw;
        }
        // CGS2 against V_0..V_j, then |w|^2 and V_{j+1} = w / |w|
        for (int pass = 0; pass < 2; ++pass) {
            const int off = pass == 0 ? H_OFF1 : H_OFF2;
            hipLaunchKernelGGL(kb_dots, dim3(vb, j + 1), dim3(TPB), 0, s, D.V, D.ld, j + 1, wv,
                               D.dpart, D.nvb);
            hipLaunchKernelGGL(kb_red, dim3(ns, j + 1), dim3(TPB), 0, s, D.dpart, D.nvb, D.sd, off,
                               D.red);
            hipLaunchKernelGGL(kb_sub_basis, dim3(vb), dim3(TPB), 0, s, D.V, D.ld, j + 1, D.red,
                               off, D.vblk2sys, wv);
        }
        hipLaunchKernelGGL(kb_dots, dim3(vb, 1), dim3(TPB), 0, s, D.V, D.ld, 0, wv, D.dpart,
                           D.nvb);
        hipLaunchKernelGGL(kb_red, dim3(ns, 1), dim3(TPB), 0, s, D.dpart, D.nvb, D.sd, H_NRM,
                           D.red);
        hipLaunchKernelGGL(kb_scale, dim3(vb), dim3(TPB), 0, s, wv, D.red, D.vblk2sys,
                           D.V + (int64_t)(j + 1) * D.ld);
        hipLaunchKernelGGL(kb_givens, dim3(sb), dim3(256), 0, s, D.st, D.red, ns, j, m, p->tol,
                           f32 ? std::max(p->inner_tol, 1e-7) : 0.0, p->max_iter, D.mask_step);
    }
    hipLaunchKernelGGL(kb_solve_y, dim3(sb), dim3(256), 0, s, D.st, ns, m);
    hipLaunchKernelGGL(kb_add_basis, dim3(vb), dim3(TPB), 0, s, D.V, D.ld, m, D.st, D.vblk2sys, x);
    // r = rhs - A x in FP64 for the systems of this cycle, then the next start
    enqueue_matvec(c, P, D, false, trans, D.mask_run, eps, kap, x, D.w);
    if (D.pc_leaves > 0) {
        hipLaunchKernelGGL(kb_axpby, dim3(vb), dim3(TPB), 0, s, rhs, D.w, -1.0, D.pw);
        pc_apply_batch(s, D, trans, D.pw, D.r);
    } else {
        hipLaunchKernelGGL(kb_axpby, dim3(vb), dim3(TPB), 0, s, rhs, D.w, -1.0, D.r);
    }
    hipLaunchKernelGGL(kb_dots, dim3(vb, 1), dim3(TPB), 0, s, D.V, D.ld, 0, D.r, D.dpart, D.nvb);
    hipLaunchKernelGGL(kb_red, dim3(ns, 1), dim3(TPB), 0, s, D.dpart, D.nvb, D.sd, H_NRM, D.red);
    hipLaunchKernelGGL(kb_begin, dim3(1), dim3(256), 0, s, D.st, D.red, ns, m, p->tol,
                       p->max_iter, 0, D.mask_step, D.mask_run, D.active);
    hipLaunchKernelGGL(kb_scale, dim3(vb), dim3(TPB), 0, s, D.r, D.red, D.vblk2sys, D.V);
    LAUNCHCHK();
    return PB_OK;
}

// Solve A x = rhs (or A^T) for all systems; returns per-system stats in D.st.
int batch_gmres(pb_ctx *c, const BatchPlan &P, BatchDev &D, const pb_params *p, int trans,
                const double *rhs, double *x)
{
    hipStream_t s = c->stream;
    const int ns = P.n_sys, m = p->restart;
    const unsigned vb = (unsigned)D.nvb;
    const unsigned sb = (unsigned)((ns + 255) / 256);
    // x = 0, r = M^-1 rhs (or rhs), |r| -> bnorm, first start
    hipLaunchKernelGGL(kb_fill, dim3(vb), dim3(TPB), 0, s, x, 0.0);
    if (D.pc_leaves > 0) {
        pc_apply_batch(s, D, trans, rhs, D.pb);
        hipLaunchKernelGGL(kb_axpby, dim3(vb), dim3(TPB), 0, s, D.pb, x, 0.0, D.r);
    } else {
        hipLaunchKernelGGL(kb_axpby, dim3(vb), dim3(TPB), 0, s, rhs, x, 0.0, D.r);
    }
    hipLaunchKernelGGL(kb_dots, dim3(vb, 1), dim3(TPB), 0, s, D.V, D.ld, 0, D.r, D.dpart, D.nvb);
    hipLaunchKernelGGL(kb_red, dim3(ns, 1), dim3(TPB), 0, s, D.dpart, D.nvb, D.sd, H_NRM, D.red);
    hipLaunchKernelGGL(kb_init, dim3(sb), dim3(256), 0, s, D.st, D.red, ns);
    hipLaunchKernelGGL(kb_begin, dim3(1), dim3(256), 0, s, D.st, D.red, ns, m, p->tol, p->max_iter,
                       1, D.mask_step, D.mask_run, D.active);
    hipLaunchKernelGGL(kb_scale, dim3(vb), dim3(TPB), 0, s, D.r, D.red, D.vblk2sys, D.V);
    LAUNCHCHK();
    // capture one cycle
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_cycle(c, P, D, p, trans, rhs, x);
    hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc < 0) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return rc;
    }
    HIPCHK(ec);
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(ec);
    const int max_cycles = p->max_iter / std::max(1, m) + 2;
    int status = PB_OK;
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        ec = hipGraphLaunch(exec, s);
        if (ec != hipSuccess) {
            status = fail(c, PB_ERR_HIP, "hipGraphLaunch failed: %s", hipGetErrorString(ec));
            break;
        }
        int32_t act = 0;
        ec = hipMemcpyAsync(&act, D.active, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (ec == hipSuccess)
            ec = hipStreamSynchronize(s);
        if (ec != hipSuccess) {
            status = fail(c, PB_ERR_HIP, "graph replay failed: %s", hipGetErrorString(ec));
            break;
        }
        if (act == 0)
            break;
    }
    (void)hipGraphExecDestroy(exec);
    return status;
}

int upload(pb_ctx *c, void *dst, const void *src, size_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    return PB_OK;
}

// Batched FP32 forward sweep over all systems timed for each candidate
// configuration (HIP events, one warm-up and three timed launches each); the
// fastest is kept in the context.
int batch_tune_run(pb_ctx *c, BatchPlan &P, BatchDev &D, const pb_params *p, BatchTune &tn)
{
    hipStream_t s = c->stream;
    const int ns = P.n_sys;
    const double eps = p->eps_out / p->eps_in, kap = p->kappa;
    {
        std::vector<int32_t> ones(ns, 1);
        TRY(upload(c, D.mask_step, ones.data(), sizeof(int32_t) * ns));
    }
    hipLaunchKernelGGL(kb_fill, dim3((unsigned)D.nvb), dim3(TPB), 0, s, D.x, 1.0);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(s));
    const int kind0 = c->f32_tpt, tiles0 = c->b_sym_tiles;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best = -1;
    int rc = PB_OK;
    for (int k = 0; k < tn.n && rc == PB_OK; ++k) {
        c->f32_tpt = tn.kind[k];
        if (tn.kind[k] == PB_SWEEP_PAIRWISE) {
            plan_sym_items(P, tn.tiles[k]);
            rc = ensure(c, c->b_sitems, sizeof(SItem) * std::max<size_t>(P.sitems.size(), 1));
            if (rc == PB_OK)
                rc = ensure(c, c->b_srow,
                            sizeof(double) * 2 * TILE * std::max<int64_t>(P.n_slots, 1));
            if (rc != PB_OK)
                break;
            D.sitems = as<SItem>(c->b_sitems);
            D.srow = as<double>(c->b_srow);
            if (hipMemcpyAsync(D.sitems, P.sitems.data(), sizeof(SItem) * P.sitems.size(),
                               hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(D.rs, P.rs.data(), sizeof(int32_t) * P.rs.size(),
                               hipMemcpyHostToDevice, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = fail(c, PB_ERR_HIP, "autotune upload failed");
                break;
            }
        }
        enqueue_matvec(c, P, D, true, 0, D.mask_step, eps, kap, D.x, D.w);
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r)
            enqueue_matvec(c, P, D, true, 0, D.mask_step, eps, kap, D.x, D.w);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(c, PB_ERR_HIP, "autotune launch failed: %s",
                      hipGetErrorString(hipGetLastError()));
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        tn.ms[k] = ms / 3.0;
        if (best < 0 || tn.ms[k] < tn.ms[best])
            best = k;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PB_OK || best < 0) {
        c->f32_tpt = kind0;
        c->b_sym_tiles = tiles0;
        return rc != PB_OK ? rc : fail(c, PB_ERR_ARG, "no autotune candidate");
    }
    c->f32_tpt = tn.kind[best];
    if (tn.kind[best] == PB_SWEEP_PAIRWISE)
        c->b_sym_tiles = tn.tiles[best];
    tn.best = best;
    return PB_OK;
}

}  // namespace

int batch_solve(pb_ctx *c, int32_t n_sys, const pb_surface *surf, const pb_charges *chg,
                const pb_params *p, int want_forces, double *e_solv, double *dE_dpos,
                double *dE_dq, pb_info *info, BatchTune *tune, bool device_inputs)
{
    if (n_sys < 1 || !surf || !chg || (!e_solv && !tune))
        return fail(c, PB_ERR_ARG, "batch needs n_sys >= 1, surfaces, charges and e_solv");
    if (p->restart > BM_MAX)
        return fail(c, PB_ERR_ARG, "batched solves support restart <= %d", BM_MAX);
    if (want_forces && (!dE_dpos || !dE_dq))
        return fail(c, PB_ERR_ARG, "gradient outputs are NULL");
    for (int b = 0; b < n_sys; ++b) {
        if (!surf[b].vert || !surf[b].tri || surf[b].n_tri <= 0 || surf[b].n_vert < 3)
            return fail(c, PB_ERR_ARG, "system %d: bad surface arguments", b);
        if (!chg[b].pos || !chg[b].q || chg[b].n <= 0)
            return fail(c, PB_ERR_ARG, "system %d: bad charge arguments", b);
    }
    hipStream_t s = c->stream;
    BatchPlan P;
    plan_batch(P, n_sys, surf, chg, c->b_sym_tiles);
    BatchDev D;
    const int m = p->restart;
    D.vtot = 2 * P.gtot;
    D.nvb = D.vtot / TPB;
    D.ld = D.vtot;
    const int64_t ni = (int64_t)P.items.size(), nci = (int64_t)P.citems.size();
    // device memory (reused across calls through the context's buffers)
    TRY(ensure(c, c->b_geo, sizeof(double) * 7 * P.gtot));
    TRY(ensure(c, c->b_desc, sizeof(SysDesc) * n_sys + sizeof(GState) * n_sys +
                                 sizeof(int32_t) * (4 * n_sys + 64)));
    TRY(ensure(c, c->b_map, sizeof(int32_t) * (P.blk2sys.size() + P.vblk2sys.size() +
                                               P.cblk2sys.size())));
    TRY(ensure(c, c->b_items, sizeof(Item) * (ni + nci)));
    TRY(ensure(c, c->b_src, sizeof(double) * 16 * P.gtot));
    TRY(ensure(c, c->b_sitems, sizeof(SItem) * std::max<size_t>(P.sitems.size(), 1)));
    TRY(ensure(c, c->b_rs, sizeof(int32_t) * P.rs.size()));
    TRY(ensure(c, c->b_srow, sizeof(double) * 2 * TILE * std::max<int64_t>(P.n_slots, 1)));
    TRY(ensure(c, c->b_scol, sizeof(double) * 2 * TILE * std::max<int64_t>(P.cptot, 1)));
    TRY(ensure(c, c->b_part, sizeof(double) * TPB * std::max<int64_t>(2 * ni, 8 * nci)));
    TRY(ensure(c, c->b_vec, sizeof(double) * 8 * D.vtot));
    TRY(ensure(c, c->b_V, sizeof(double) * (m + 1) * D.vtot));
    TRY(ensure(c, c->b_red, sizeof(double) * ((int64_t)HB * n_sys + (int64_t)(m + 2) * D.nvb +
                                              8 * P.ctot + n_sys)));
    TRY(ensure(c, c->b_chg, sizeof(double) * 4 * P.ctot));
    D.g = as<double>(c->b_geo);
    char *dp = static_cast<char *>(c->b_desc.p);
    D.sd = reinterpret_cast<SysDesc *>(dp);
    D.st = reinterpret_cast<GState *>(dp + sizeof(SysDesc) * n_sys);
    int32_t *ip = reinterpret_cast<int32_t *>(dp + sizeof(SysDesc) * n_sys + sizeof(GState) * n_sys);
    D.mask_step = ip;
    D.mask_run = ip + n_sys;
    D.active = ip + 2 * n_sys;
    int32_t *mp = as<int32_t>(c->b_map);
    D.blk2sys = mp;
    D.vblk2sys = mp + P.blk2sys.size();
    D.cblk2sys = D.vblk2sys + P.vblk2sys.size();
    D.items = as<Item>(c->b_items);
    D.citems = D.items + ni;
    D.src = c->b_src.p;
    D.sitems = as<SItem>(c->b_sitems);
    D.rs = as<int32_t>(c->b_rs);
    D.srow = as<double>(c->b_srow);
    D.scol = c->b_scol.p;
    D.part = as<double>(c->b_part);
    double *vp = as<double>(c->b_vec);
    D.x = vp;
    D.b = vp + D.vtot;
    D.w = vp + 2 * D.vtot;
    D.r = vp + 3 * D.vtot;
    D.t = vp + 4 * D.vtot;
    D.lam = vp + 5 * D.vtot;
    D.pw = vp + 6 * D.vtot;
    D.pb = vp + 7 * D.vtot;
    D.V = as<double>(c->b_V);
    D.red = as<double>(c->b_red);
    D.dpart = D.red + (int64_t)HB * n_sys;
    D.per = D.dpart + (int64_t)(m + 2) * D.nvb;
    D.e = D.per + 8 * P.ctot;
    D.pos = as<double>(c->b_chg);
    D.q = D.pos + 3 * P.ctot;

    // geometry of every system (validated), then centres
    int64_t max_nv = 0, max_nt = 0;
    for (int b = 0; b < n_sys; ++b) {
        max_nv = std::max<int64_t>(max_nv, surf[b].n_vert);
        max_nt = std::max<int64_t>(max_nt, surf[b].n_tri);
    }
    const int gblk = geometry_blocks(round_up(max_nt, PADN));
    TRY(ensure(c, c->in_vert, sizeof(double) * 3 * max_nv));
    TRY(ensure(c, c->in_tri, sizeof(int32_t) * 3 * max_nt));
    TRY(ensure(c, c->geo_part, sizeof(double) * GEO_RED * gblk));
    TRY(ensure(c, c->small, sizeof(double) * HSMALL));
    const int64_t dcap = dup_table_size(max_nt);
    TRY(ensure(c, c->dup_tab, sizeof(int32_t) * (dcap + 2)));
    int32_t *hdup = reinterpret_cast<int32_t *>(c->hsmall + HSMALL_DUP);
    double max_len = 0.0;
    for (int b = 0; b < n_sys; ++b) {
        SysDesc &d = P.sd[b];
        const double *dv = surf[b].vert;
        const int32_t *dt = surf[b].tri;
        if (!device_inputs) {
            TRY(upload(c, c->in_vert.p, surf[b].vert, sizeof(double) * 3 * surf[b].n_vert));
            TRY(upload(c, c->in_tri.p, surf[b].tri, sizeof(int32_t) * 3 * surf[b].n_tri));
            dv = as<double>(c->in_vert);
            dt = as<int32_t>(c->in_tri);
        }
        const int nb = geometry_blocks(d.npad);
        launch_geometry(s, surf[b].n_vert, d.n, dv, dt, D.g + d.goff, d.npad, P.gtot,
                        as<double>(c->geo_part), nb);
        launch_reduce_cols(s, as<double>(c->geo_part), nb, GEO_RED, as<double>(c->small));
        LAUNCHCHK();
        launch_dup_check(s, D.g + d.goff, d.n, P.gtot, as<int32_t>(c->dup_tab), dcap);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(c->hsmall, c->small.p, sizeof(double) * GEO_RED,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hdup, as<int32_t>(c->dup_tab) + dcap, sizeof(int32_t) * 2,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double *r = c->hsmall;
        if (r[0] != 0.0)
            return fail(c, PB_ERR_GEOMETRY, "system %d: %.0f bad triangle(s)", b, r[0]);
        if (r[6] != 0.0)
            return fail(c, PB_ERR_GEOMETRY,
                        "system %d: %.0f triangle(s) with a centroid coordinate beyond %g A", b,
                        r[6], COORD_MAX);
        if (hdup[1] != 0)
            return fail(c, PB_ERR_GEOMETRY,
                        "system %d: triangle %d shares its centroid with another triangle", b,
                        hdup[0]);
        if (!(r[1] > 0.0))
            return fail(c, PB_ERR_GEOMETRY, "system %d: non-positive enclosed volume", b);
        max_len = std::max(max_len, std::sqrt(r[5] / (2.0 * TWO_PI)));
        d.cx = r[2] / (double)d.n;
        d.cy = r[3] / (double)d.n;
        d.cz = r[4] / (double)d.n;
    }
    P.sigma_min = 1.0 / max_len;
    // charges, padded per system (padding repeats the last charge with q = 0)
    {
        std::vector<double> hp, hq;
        if (device_inputs) {
            for (int b = 0; b < n_sys; ++b) {
                const SysDesc &d = P.sd[b];
                HIPCHK(hipMemcpyAsync(D.pos + 3 * d.coff, chg[b].pos, sizeof(double) * 3 * d.nc,
                                      hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(D.q + d.coff, chg[b].q, sizeof(double) * d.nc,
                                      hipMemcpyDeviceToDevice, s));
            }
        } else {
            hp.assign(3 * P.ctot, 0.0);
            hq.assign(P.ctot, 0.0);
            for (int b = 0; b < n_sys; ++b) {
                const SysDesc &d = P.sd[b];
                for (int64_t k = 0; k < d.nc; ++k) {
                    for (int e = 0; e < 3; ++e)
                        hp[3 * (d.coff + k) + e] = chg[b].pos[3 * k + e];
                    hq[d.coff + k] = chg[b].q[k];
                }
            }
            TRY(upload(c, D.pos, hp.data(), sizeof(double) * 3 * P.ctot));
            TRY(upload(c, D.q, hq.data(), sizeof(double) * P.ctot));
        }
        TRY(upload(c, D.sd, P.sd.data(), sizeof(SysDesc) * n_sys));
        hipLaunchKernelGGL(kb_pad_charges, dim3(n_sys), dim3(TPB), 0, s, D.sd, D.pos, D.q);
        LAUNCHCHK();
        TRY(upload(c, D.blk2sys, P.blk2sys.data(), sizeof(int32_t) * P.blk2sys.size()));
        TRY(upload(c, D.vblk2sys, P.vblk2sys.data(), sizeof(int32_t) * P.vblk2sys.size()));
        TRY(upload(c, D.cblk2sys, P.cblk2sys.data(), sizeof(int32_t) * P.cblk2sys.size()));
        TRY(upload(c, D.items, P.items.data(), sizeof(Item) * ni));
        TRY(upload(c, D.citems, P.citems.data(), sizeof(Item) * nci));
        if (!P.sitems.empty())
            TRY(upload(c, D.sitems, P.sitems.data(), sizeof(SItem) * P.sitems.size()));
        TRY(upload(c, D.rs, P.rs.data(), sizeof(int32_t) * P.rs.size()));
        HIPCHK(hipStreamSynchronize(s));   // host staging vectors go out of scope
    }
    if (tune)
        return batch_tune_run(c, P, D, p, *tune);
    const double eps = p->eps_out / p->eps_in, kap = p->kappa;
    const unsigned gb = nblk(P.gtot), vb = (unsigned)D.nvb, cbk = nblk(P.ctot);
    // preconditioned vectors: the apply writes real entries only, so the
    // padding of these two must start (and stay) zero
    hipLaunchKernelGGL(kb_fill, dim3(vb), dim3(TPB), 0, s, D.pw, 0.0);
    hipLaunchKernelGGL(kb_fill, dim3(vb), dim3(TPB), 0, s, D.pb, 0.0);
    LAUNCHCHK();
    if (p->precond_leaf > 0) {
        // centroids of every system (3 gtot doubles, one copy) into pinned staging
        if (c->hgeo_n < (size_t)(3 * P.gtot)) {
            if (c->hgeo)
                (void)hipHostFree(c->hgeo);
            c->hgeo = nullptr;
            c->hgeo_n = 0;
            if (hipHostMalloc(reinterpret_cast<void **>(&c->hgeo), sizeof(double) * 3 * P.gtot,
                              hipHostMallocDefault) != hipSuccess)
                return fail(c, PB_ERR_OOM, "pinned host staging of %lld doubles",
                            (long long)(3 * P.gtot));
            c->hgeo_n = (size_t)(3 * P.gtot);
        }
        const double *hg = c->hgeo;
        HIPCHK(hipMemcpyAsync(c->hgeo, D.g, sizeof(double) * 3 * P.gtot, hipMemcpyDeviceToHost,
                              s));
        HIPCHK(hipStreamSynchronize(s));
        // the systems' octrees are independent: built side by side by a few
        // workers (each tree single-threaded), joined in system order
        std::vector<std::vector<int32_t>> sperm(n_sys), sstart(n_sys);
        {
            std::atomic<int> next{0};
            auto work = [&] {
                for (int b = next++; b < n_sys; b = next++) {
                    const SysDesc &d = P.sd[b];
                    build_leaves(hg + d.goff, hg + P.gtot + d.goff, hg + 2 * P.gtot + d.goff, d.n,
                                 p->precond_leaf, sperm[b], sstart[b], false);
                }
            };
            const unsigned hw = std::thread::hardware_concurrency();
            const int nw = (int)std::min<unsigned>(std::max(1u, hw ? hw : 1u), 16u) - 1;
            std::vector<std::thread> pool;
            for (int k = 0; k < std::min(nw, n_sys - 1); ++k) {
                try {
                    pool.emplace_back(work);
                } catch (const std::system_error &) {
                    break;   // fewer workers; the calling thread works too
                }
            }
            work();
            for (auto &t : pool)
                t.join();
        }
        std::vector<int32_t> gperm, gstart(1, 0);
        std::vector<int64_t> gboff(1, 0);
        std::vector<int64_t> sbase(n_sys + 1, 0);   // first element of each system in gperm
        for (int b = 0; b < n_sys; ++b) {
            const SysDesc &d = P.sd[b];
            const std::vector<int32_t> &perm = sperm[b], &start = sstart[b];
            const int32_t base = (int32_t)gperm.size();
            sbase[b] = base;
            for (int32_t e : perm)
                gperm.push_back((int32_t)(d.goff + e));
            for (size_t l = 1; l < start.size(); ++l) {
                gstart.push_back(base + start[l]);
                const int64_t m2 = 2 * (int64_t)(start[l] - start[l - 1]);
                gboff.push_back(gboff.back() + m2 * m2);
            }
        }
        sbase[n_sys] = (int64_t)gperm.size();
        const int64_t L = (int64_t)gstart.size() - 1, ne = (int64_t)gperm.size();
        const size_t off64 = round_up(sizeof(int32_t) * (ne + L + 1), 8);
        TRY(ensure(c, c->b_pc_idx, off64 + sizeof(int64_t) * (L + 1 + 2 * ne)));
        TRY(ensure(c, c->b_pc_inv, sizeof(double) * std::max<int64_t>(gboff.back(), 1)));
        D.pc_perm = as<int32_t>(c->b_pc_idx);
        D.pc_start = D.pc_perm + ne;
        D.pc_boff = reinterpret_cast<int64_t *>(static_cast<char *>(c->b_pc_idx.p) + off64);
        D.pc_pidx = D.pc_boff + (L + 1);
        D.pc_qidx = D.pc_pidx + ne;
        D.pc_inv = as<double>(c->b_pc_inv);
        TRY(upload(c, D.pc_perm, gperm.data(), sizeof(int32_t) * ne));
        TRY(upload(c, D.pc_start, gstart.data(), sizeof(int32_t) * (L + 1)));
        TRY(upload(c, D.pc_boff, gboff.data(), sizeof(int64_t) * (L + 1)));
        // phi and psi slots of every element, from its system's layout
        TRY(ensure(c, c->b_pc_sys, sizeof(int64_t) * (n_sys + 1)));
        TRY(upload(c, c->b_pc_sys.p, sbase.data(), sizeof(int64_t) * (n_sys + 1)));
        hipLaunchKernelGGL(kb_pc_index, dim3(nblk(ne)), dim3(TPB), 0, s, D.pc_perm, ne,
                           as<int64_t>(c->b_pc_sys), D.sd, n_sys, D.pc_pidx, D.pc_qidx);
        LAUNCHCHK();
        Geo gall;
        gall.g = D.g;
        gall.n = P.gtot;
        gall.npad = P.gtot;   // array stride of the concatenated geometry
        launch_pc_build(s, gall, D.pc_perm, D.pc_start, D.pc_boff, L, p->precond_leaf, eps, kap,
                        D.pc_inv);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(s));   // host index vectors go out of scope
        D.pc_leaves = L;
    }
    const unsigned cgrid = item_grid(nci);
    // charges inside: solid angle with phi = 1, psi = 0
    {
        hipLaunchKernelGGL(kb_fill, dim3(vb), dim3(TPB), 0, s, D.t, 0.0);
        // phi = 1 on real entries: pack reads phi from the vector; set it by a fill of the
        // first halves through the geometry (area 0 on padding makes padding inert)
        std::vector<double> ones(D.vtot, 0.0);
        for (int b = 0; b < n_sys; ++b)
            for (int64_t j = 0; j < P.sd[b].n; ++j)
                ones[2 * P.sd[b].goff + j] = 1.0;
        TRY(upload(c, D.t, ones.data(), sizeof(double) * D.vtot));
        hipLaunchKernelGGL(kb_pack<double>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, D.t, reinterpret_cast<Src8<double> *>(D.src), 0, eps);
        hipLaunchKernelGGL(kb_charge_pairs<1>, dim3(cgrid), dim3(TPB), 0, s,
                           reinterpret_cast<const Src8<double> *>(D.src), nullptr, D.sd, D.citems,
                           nci, D.pos, eps, kap, D.part);
        hipLaunchKernelGGL(kb_charge_sum<1>, dim3(cbk), dim3(TPB), 0, s, D.part, nci, D.sd,
                           D.cblk2sys, D.per);
        LAUNCHCHK();
        std::vector<double> om(P.ctot);
        HIPCHK(hipMemcpyAsync(om.data(), D.per, sizeof(double) * P.ctot, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int b = 0; b < n_sys; ++b)
            for (int64_t k = 0; k < P.sd[b].nc; ++k)
                if (!(om[P.sd[b].coff + k] >= 2.0 * M_PI))
                    return fail(c, PB_ERR_CHARGE, "system %d: charge %lld is not inside the surface",
                                b, (long long)k);
    }
    // sources
    hipLaunchKernelGGL(kb_source, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd, D.blk2sys, D.pos,
                       D.q, INV_4PI / p->eps_in, 0, eps, kap, D.b);
    LAUNCHCHK();
    TRY(batch_gmres(c, P, D, p, 0, D.b, D.x));
    std::vector<GState> hst(n_sys);
    HIPCHK(hipMemcpyAsync(hst.data(), D.st, sizeof(GState) * n_sys, hipMemcpyDeviceToHost, s));
    // energy
    hipLaunchKernelGGL(kb_pack<double>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd, D.blk2sys,
                       D.x, reinterpret_cast<Src8<double> *>(D.src), 0, eps);
    std::vector<GState> ast;
    if (!want_forces) {
        hipLaunchKernelGGL(kb_charge_pairs<0>, dim3(cgrid), dim3(TPB), 0, s,
                           reinterpret_cast<const Src8<double> *>(D.src), nullptr, D.sd, D.citems,
                           nci, D.pos, eps, kap, D.part);
        hipLaunchKernelGGL(kb_charge_sum<1>, dim3(cbk), dim3(TPB), 0, s, D.part, nci, D.sd,
                           D.cblk2sys, D.per);
        hipLaunchKernelGGL(kb_energy, dim3(n_sys), dim3(TPB), 0, s, D.per, 1, D.q, D.sd,
                           0.5 * 332.0716, D.e);
        LAUNCHCHK();
    } else {
        // adjoint: A^T lam' = B'^T q, then the gradient sweep
        hipLaunchKernelGGL(kb_source, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd, D.blk2sys,
                           D.pos, D.q, 0.0, 1, eps, kap, D.t);
        LAUNCHCHK();
        TRY(batch_gmres(c, P, D, p, 1, D.t, D.lam));
        ast.resize(n_sys);
        HIPCHK(hipMemcpyAsync(ast.data(), D.st, sizeof(GState) * n_sys, hipMemcpyDeviceToHost, s));
        double *fwd = static_cast<double *>(D.src);
        double *adj = fwd + 8 * P.gtot;
        hipLaunchKernelGGL(kb_pack<double>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, D.x, reinterpret_cast<Src8<double> *>(fwd), 0, eps);
        hipLaunchKernelGGL(kb_pack<double>, dim3(gb), dim3(TPB), 0, s, D.g, P.gtot, D.sd,
                           D.blk2sys, D.lam, reinterpret_cast<Src8<double> *>(adj), 1, eps);
        hipLaunchKernelGGL(kb_charge_pairs<2>, dim3(cgrid), dim3(TPB), 0, s,
                           reinterpret_cast<const Src8<double> *>(fwd),
                           reinterpret_cast<const Src8<double> *>(adj), D.sd, D.citems, nci, D.pos,
                           eps, kap, D.part);
        hipLaunchKernelGGL(kb_charge_sum<8>, dim3(cbk), dim3(TPB), 0, s, D.part, nci, D.sd,
                           D.cblk2sys, D.per);
        hipLaunchKernelGGL(kb_energy, dim3(n_sys), dim3(TPB), 0, s, D.per, 8, D.q, D.sd,
                           0.5 * 332.0716, D.e);
        // caller host arrays are filled through device staging, device arrays directly
        int64_t nct = 0;
        for (int b = 0; b < n_sys; ++b)
            nct += P.sd[b].nc;
        double *gpos = dE_dpos, *gq = dE_dq;
        if (!device_inputs) {
            TRY(ensure(c, c->io_y, sizeof(double) * 4 * nct));
            gpos = as<double>(c->io_y);
            gq = gpos + 3 * nct;
        }
        hipLaunchKernelGGL(kb_force_out, dim3(cbk), dim3(TPB), 0, s, D.per, D.q, D.sd, D.cblk2sys,
                           0.5 * 332.0716, 1.0 / (4.0 * M_PI * p->eps_in), gpos, gq);
        LAUNCHCHK();
        if (!device_inputs) {
            HIPCHK(hipMemcpyAsync(dE_dpos, gpos, sizeof(double) * 3 * nct, hipMemcpyDeviceToHost,
                                  s));
            HIPCHK(hipMemcpyAsync(dE_dq, gq, sizeof(double) * nct, hipMemcpyDeviceToHost, s));
        }
    }
    HIPCHK(hipMemcpyAsync(e_solv, D.e, sizeof(double) * n_sys, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int status = PB_OK;
    for (int b = 0; b < n_sys; ++b) {
        const GState &f = hst[b];
        int st = f.conv ? PB_OK : PB_NOT_CONVERGED;
        if (want_forces && !ast[b].conv)
            st = PB_NOT_CONVERGED;
        if (st != PB_OK)
            status = PB_NOT_CONVERGED;
        if (info) {
            pb_info &o = info[b];
            o.e_solv = e_solv[b];
            o.rel_residual = f.rel;
            o.seconds = 0.0;
            o.iters = f.iters;
            const int arn = f.iters + (want_forces ? ast[b].iters : 0);
            const int res = f.nres + (want_forces ? ast[b].nres : 0);
            o.matvecs_fp32 = p->precision == PB_FP32_IR ? arn : 0;
            o.matvecs_fp64 = (p->precision == PB_FP32_IR ? 0 : arn) + res;
            o.refinements = p->precision == PB_FP32_IR ? f.nres : 0;
            o.status = st;
            o.adjoint_iters = want_forces ? ast[b].iters : 0;
        }
    }
    if (status == PB_NOT_CONVERGED)
        fail(c, PB_NOT_CONVERGED, "some systems of the batch did not reach tol %.3e", p->tol);
    return status;
}

}  // namespace pbk
