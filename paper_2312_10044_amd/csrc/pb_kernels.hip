// HIP kernels (gfx950) of the DSBI Poisson-Boltzmann path.
//
// Pair sweeps (matvec, its transpose, sources, reaction potential) are
// O(N^2) / O(N Nc) n-body sums: each thread keeps one target in registers,
// the block stages a tile of TILE packed sources in LDS with coalesced
// loads, and every lane reads the same LDS entry (broadcast, conflict free)
// while walking the tile.  The source range is split into chunks so that a
// launch holds ~10 waves per SIMD; chunk = blockIdx % n_chunks keeps each
// XCD's blocks on the same sources (blocks are dealt to the 8 XCDs round
// robin), so each XCD's L2 holds only its own share of the stream.  Chunk
// partials are summed in a fixed order by a second kernel: results are
// bitwise reproducible.  No atomics anywhere.
//
// Kernel algebra (collocation pair i <- j, d = x_i - x_j, r = |d|,
// e = exp(-kappa r), tm1 = (1 + kappa r) e - 1, eps = eps_out/eps_in,
// c_x = n_i.d, u = 1/r^3; the 1/(4 pi) is applied once per row):
//   4pi K1 = (1 - e)/r
//   4pi K2 = (eps (1 + kappa r) e - 1) (n_j.d) u
//   4pi K3 = ((1 + kappa r) e / eps - 1) c_x u
//   4pi K4 = u [tm1 (n_i.n_j) - c_x (n_j.d) (3 tm1 / r^2 + kappa^2 e)]
// These are the kernels of eqs. Eq_K1/Eq_K2 with d/dnu_x = +nu_x.grad_x
// (Sec. 2.2.1).  The source stream carries w_j = a_j psi_j and
// m_j = a_j phi_j n_j, so the per-pair work needs no separate phi_j, n_j:
//   row 1: sum_j [-(e-1)/r w_j + g2 (m_j.d) u]          g2 = eps tm1 + eps - 1
//   row 2: sum_j u [tm1 (n_i.m_j) - c_x ((m_j.d) h - g3 w_j)]
//          h = 3 tm1/r^2 + kappa^2 e,  g3 = tm1/eps + 1/eps - 1
// The transpose swaps the roles: w_j = l1_j, m_j = l2_j n_j and
//   row 1: sum_j u [tm1 (n_i.m_j) - c_x ((m_j.d) h + g2 w_j)]
//   row 2: sum_j [-(e-1)/r w_j - g3 (m_j.d) u]
// with the target area a_i applied once per row.
#include "pb_kernels.h"
#include "pb_device.h"

#include <algorithm>

#include <cmath>

namespace pbk {

namespace {

using namespace dev;

// ---- geometry -------------------------------------------------------------

__global__ __launch_bounds__(TPB) void k_geometry(int64_t n_vert, int64_t n_tri,
                                                  const double *__restrict__ vert,
                                                  const int32_t *__restrict__ tri,
                                                  double *__restrict__ g, int64_t npad,
                                                  int64_t ld, double *__restrict__ part, int nblk)
{
#pragma clang fp contract(off)
    __shared__ double sh[TPB / 64];
    double acc[GEO_RED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < npad;
         i += (int64_t)gridDim.x * TPB) {
        double c[3] = {FAR_TGT, 0.0, 0.0}, nn[3] = {0.0, 0.0, 1.0}, a = 0.0;
        if (i < n_tri) {
            const int32_t ia = tri[3 * i], ib = tri[3 * i + 1], ic = tri[3 * i + 2];
            bool bad = ia < 0 || ib < 0 || ic < 0 || ia >= n_vert || ib >= n_vert || ic >= n_vert;
            if (!bad) {
                const double *v0 = vert + 3 * (int64_t)ia;
                const double *v1 = vert + 3 * (int64_t)ib;
                const double *v2 = vert + 3 * (int64_t)ic;
                double e1[3], e2[3], m[3];
                for (int k = 0; k < 3; ++k) {
                    c[k] = (v0[k] + v1[k] + v2[k]) / 3.0;
                    e1[k] = v1[k] - v0[k];
                    e2[k] = v2[k] - v0[k];
                }
                m[0] = e1[1] * e2[2] - e1[2] * e2[1];
                m[1] = e1[2] * e2[0] - e1[0] * e2[2];
                m[2] = e1[0] * e2[1] - e1[1] * e2[0];
                const double mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
                a = 0.5 * mn;
                for (int k = 0; k < 3; ++k)
                    nn[k] = m[k] / mn;
                const double chk = c[0] + c[1] + c[2] + nn[0] + nn[1] + nn[2] + a;
                bad = !(mn > 0.0) || !isfinite(chk);
                if (!bad && !(fabs(c[0]) <= COORD_MAX && fabs(c[1]) <= COORD_MAX &&
                              fabs(c[2]) <= COORD_MAX)) {
                    bad = true;   // counted apart, for a message of its own
                    acc[6] += 1.0;
                    acc[0] -= 1.0;
                }
                if (!bad) {
                    acc[1] += m[0] * c[0] + m[1] * c[1] + m[2] * c[2];
                    acc[2] += c[0];
                    acc[3] += c[1];
                    acc[4] += c[2];
                    acc[5] += a;
                }
            }
            if (bad) {
                acc[0] += 1.0;
                c[0] = FAR_TGT; c[1] = 0.0; c[2] = 0.0;
                nn[0] = 0.0; nn[1] = 0.0; nn[2] = 1.0;
                a = 0.0;
            }
        }
        g[i] = c[0];
        g[ld + i] = c[1];
        g[2 * ld + i] = c[2];
        g[3 * ld + i] = nn[0];
        g[4 * ld + i] = nn[1];
        g[5 * ld + i] = nn[2];
        g[6 * ld + i] = a;
    }
    for (int k = 0; k < GEO_RED; ++k) {
        const double s = block_sum(acc[k], sh);
        if (threadIdx.x == 0)
            part[(int64_t)k * nblk + blockIdx.x] = s;
    }
}

// ---- coincident collocation points ------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(TPB) void k_dup_clear(int32_t *__restrict__ tab, int64_t cap)
{
    for (int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x; k < cap + 2;
         k += (int64_t)gridDim.x * TPB)
        tab[k] = k < cap ? -1 : (k == cap ? INT32_MAX : 0);
}

// Open-addressing insert of every centroid, keyed by its coordinates (+0.0
// folds -0 into 0).  Points with equal centroids probe the same slots, so each
// one after the first to claim a slot finds that first one; the smallest index
// over these pairs is the smallest index of any coincident group, whichever
// point won.  The table holds >= 2n slots and at most n entries, so every
// probe sequence reaches an empty slot.
__global__ __launch_bounds__(TPB) void k_dup_insert(const double *__restrict__ g, int64_t n,
                                                    int64_t ld, int32_t *__restrict__ tab,
                                                    int64_t cap)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n || !(g[6 * ld + i] > 0.0))
        return;
    const double x = g[i] + 0.0, y = g[ld + i] + 0.0, z = g[2 * ld + i] + 0.0;
    const uint64_t h = mix64((uint64_t)__double_as_longlong(x) ^
                             mix64((uint64_t)__double_as_longlong(y) ^
                                   mix64((uint64_t)__double_as_longlong(z))));
    const uint64_t mask = (uint64_t)cap - 1;
    int32_t *out = tab + cap;
    for (uint64_t slot = h & mask;; slot = (slot + 1) & mask) {
        const int32_t prev = atomicCAS(&tab[slot], -1, (int32_t)i);
        if (prev < 0)
            return;
        if (g[prev] == x && g[ld + prev] == y && g[2 * ld + prev] == z) {
            atomicMin(&out[0], prev < (int32_t)i ? prev : (int32_t)i);
            atomicAdd(&out[1], 1);
            return;
        }
    }
}

// ---- packing of the source stream ---------------------------------------

template <typename T>
__global__ __launch_bounds__(TPB) void k_pack(const double *__restrict__ g, int64_t n,
                                              int64_t npad, const double *__restrict__ x,
                                              Src8<T> *__restrict__ src, int mode, double cx,
                                              double cy, double cz, double eps, double sigma)
{
    const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (j >= npad)
        return;
    Src8<T> s;
    if (j < n) {
        const double a = g[6 * npad + j];
        double w, f;
        double pad = 0.0;
        if (mode == 0) {
            w = a * x[n + j];   // a_j psi_j
            f = a * x[j];       // a_j phi_j
        } else if (mode == 1) {
            w = x[j];           // l1_j
            f = x[n + j];       // l2_j
        } else {
            const double ap = a * x[n + j] / sigma;
            w = (1.0 - 1.0 / eps) * ap;   // w1
            pad = -ap / eps;              // w2n
            f = -3.0 * a * x[j];
        }
        s.x = T((g[j] - cx) * sigma);
        s.y = T((g[npad + j] - cy) * sigma);
        s.z = T((g[2 * npad + j] - cz) * sigma);
        s.w = T(w);
        s.mx = T(f * g[3 * npad + j]);
        s.my = T(f * g[4 * npad + j]);
        s.mz = T(f * g[5 * npad + j]);
        s.pad = T(pad);
    } else {
        s.x = T((FAR_SRC - cx) * sigma);
        s.y = T(0.0);
        s.z = T(0.0);
        s.w = s.mx = s.my = s.mz = T(0.0);
        s.pad = T(0.0);
    }
    src[j] = s;
}

// ---- matvec pair sweep ----------------------------------------------------

template <typename T, bool TRANS>
__global__ __launch_bounds__(TPB) void k_pairs(const Src8<T> *__restrict__ src,
                                               const double *__restrict__ g, int64_t npad,
                                               Sweep sw, PairParams pp,
                                               double *__restrict__ part)
{
    __shared__ Src8<T> sh[TILE];
    const int b = blockIdx.x;
    const int chunk = b % sw.n_chunks;
    const int tb = b / sw.n_chunks;
    const int64_t i = (int64_t)tb * TPB + threadIdx.x;
    const T xi = T(g[i] - pp.cx), yi = T(g[npad + i] - pp.cy), zi = T(g[2 * npad + i] - pp.cz);
    const T nxi = T(g[3 * npad + i]), nyi = T(g[4 * npad + i]), nzi = T(g[5 * npad + i]);
    const Coef<T> cf(pp);
    Acc<T> aP, aQ;
    const int t0 = chunk * sw.tiles_per_chunk;
    const int t1 = min(sw.n_tiles, t0 + sw.tiles_per_chunk);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
        sh[threadIdx.x] = src[(int64_t)t * TILE + threadIdx.x];
        __syncthreads();
        T p = T(0), q = T(0);
        if (t == tb)
            sweep_tile<T, TRANS, true>(sh, threadIdx.x, xi, yi, zi, nxi, nyi, nzi, cf, p, q);
        else
            sweep_tile<T, TRANS, false>(sh, -1, xi, yi, zi, nxi, nyi, nzi, cf, p, q);
        aP.add(p);
        aQ.add(q);
    }
    const double P = aP.value(), Q = aQ.value();
    part[(int64_t)chunk * npad + i] = TRANS ? Q : P;
    part[(int64_t)(sw.n_chunks + chunk) * npad + i] = TRANS ? P : Q;
}

template <int TPT, bool SCALED>
__global__ __launch_bounds__(TPB) void k_pairs_f32_fwd(const Src8<float> *__restrict__ src,
                                                       const double *__restrict__ g, int64_t npad,
                                                       Sweep sw, PairParams pp,
                                                       double *__restrict__ part)
{
    __shared__ Src8<float> sh[TILE];
    const int b = blockIdx.x;
    const int chunk = b % sw.n_chunks;
    const int tb = b / sw.n_chunks;
    const double sig = pp.sigma;          // FP32 length unit
    const double kap = pp.kappa / sig;    // kappa in that unit (1 when SCALED)
    float tg[TPT][9];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int64_t i = ((int64_t)tb * TPT + t) * TPB + threadIdx.x;
        tg[t][0] = float((g[i] - pp.cx) * sig);
        tg[t][1] = float((g[npad + i] - pp.cy) * sig);
        tg[t][2] = float((g[2 * npad + i] - pp.cz) * sig);
        const double nx = g[3 * npad + i], ny = g[4 * npad + i], nz = g[5 * npad + i];
        tg[t][3] = float(nx);
        tg[t][4] = float(ny);
        tg[t][5] = float(nz);
        tg[t][6] = float(-nx / 3.0);
        tg[t][7] = float(-ny / 3.0);
        tg[t][8] = float(-nz / 3.0);
    }
    CoefF32 cf;
    cf.kappa = float(kap);
    cf.kexp = float(-kap * 1.4426950408889634074);
    cf.c13 = float((1.0 - 1.0 / pp.eps) / 3.0);
    cf.k23 = float(kap * kap / 3.0);
    Acc<float> aP[TPT], aQ[TPT];
    const int t0 = chunk * sw.tiles_per_chunk;
    const int t1 = min(sw.n_tiles, t0 + sw.tiles_per_chunk);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
        sh[threadIdx.x] = src[(int64_t)t * TILE + threadIdx.x];
        __syncthreads();
        float P[TPT], Q[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k)
            P[k] = Q[k] = 0.f;
        const int ds = t - tb * TPT;   // slot whose target lies in this tile
        if (ds == 0)
            sweep_f32<TPT, 0, SCALED>(sh, tg, cf, P, Q);
        else if (TPT > 1 && ds == 1)
            sweep_f32<TPT, 1, SCALED>(sh, tg, cf, P, Q);
        else
            sweep_f32<TPT, -1, SCALED>(sh, tg, cf, P, Q);
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            aP[k].add(P[k]);
            aQ[k].add(Q[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int64_t i = ((int64_t)tb * TPT + k) * TPB + threadIdx.x;
        part[(int64_t)chunk * npad + i] = aP[k].value();
        part[(int64_t)(sw.n_chunks + chunk) * npad + i] = aQ[k].value();
    }
}

// ---- pairwise FP32 sweep -----------------------------------------------------
//
// Forward (mode 0): w1 = (1 - 1/eps) a psi / sigma, w2n = -a psi / (eps sigma),
// nu = 3 a phi.  Transposed (mode 1), x = [l1; l2]: w1 = (eps - 1) l1 / sigma,
// w2n = eps l1 / sigma, nu = 3 l2.  The generic transposed pair algebra
// (P with the coefficient -g3, Q with g2) then takes the forward reduced form
// with eps replaced by 1/eps in the constant c13 = (1 - 1/eps)/3: its first
// row sums -eps P^T and its second row Q^T, in units of 1/kappa.
__global__ __launch_bounds__(TPB) void k_pack_sym(const double *__restrict__ g, int64_t n,
                                                  int64_t npad, const double *__restrict__ x,
                                                  Src12 *__restrict__ src, double cx, double cy,
                                                  double cz, double eps, double sigma, int mode)
{
    const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (j >= npad)
        return;
    Src12 s;
    if (j < n) {
        const double a = g[6 * npad + j];
        double w1, w2n, nu;
        if (mode) {
            const double w = x[j] / sigma;
            w1 = (eps - 1.0) * w;
            w2n = eps * w;
            nu = 3.0 * x[n + j];
        } else {
            const double w = a * x[n + j] / sigma;
            w1 = (1.0 - 1.0 / eps) * w;
            w2n = -w / eps;
            nu = 3.0 * a * x[j];
        }
        const double nx = g[3 * npad + j], ny = g[4 * npad + j], nz = g[5 * npad + j];
        s.x = float((g[j] - cx) * sigma);
        s.y = float((g[npad + j] - cy) * sigma);
        s.z = float((g[2 * npad + j] - cz) * sigma);
        s.w1 = float(w1);
        s.w2n = float(w2n);
        s.nx = float(-nx);
        s.ny = float(-ny);
        s.nz = float(-nz);
        s.nu = float(nu);
    } else {
        // padding: weightless points far away, 8 apart so no two coincide
        s.x = float((FAR_SRC + 8.0 * double(j - n) - cx) * sigma);
        s.y = s.z = 0.f;
        s.w1 = s.w2n = s.nu = 0.f;
        s.nx = s.ny = s.nz = 0.f;
    }
    s.res0 = s.res1 = s.res2 = 0.f;
    src[j] = s;
}

template <bool SCALED>
__global__ __launch_bounds__(SYM_NT, SYM_MIN_WAVES) void k_pairs_f32_sym(const Src12 *__restrict__ src,
                                                       const int4 *__restrict__ items, int T,
                                                       PairParams pp,
                                                       double *__restrict__ rowpart,
                                                       float *__restrict__ colpart)
{
    __shared__ SrcTileF32 sh;
    __shared__ float colw[SYM_NT / 64][2 * TILE];
    const int4 it = items[blockIdx.x];   // (I, J0, J1, slot)
    sym_item_f32<SCALED>(src, it.x, it.y, it.z, T, coef_f32(pp.eps, pp.kappa / pp.sigma, SCALED),
                         rowpart + (int64_t)it.w * (2 * TILE), colpart, sh, colw);
}

template <bool SCALED>
__global__ __launch_bounds__(BAND_WAVES * 64) void k_pairs_f32_band(const Src12 *__restrict__ src,
                                                                   const BandItem *__restrict__ items,
                                                                   int T, PairParams pp,
                                                                   float *__restrict__ recs)
{
    __shared__ BandSmem sm;
    const BandItem it = items[blockIdx.x];
    band_item_f32<SCALED>(src, it, T, coef_f32(pp.eps, pp.kappa / pp.sigma, SCALED), recs, sm);
}

// Rows of the banded sweep: row k = K*TILE + l sums the records rec_idx
// [rec_start[K], rec_start[K+1]); as in k_sym_finish, wave w of the block's
// FIN_WAVES sums every FIN_WAVES-th record from record w on and the partial
// sums are added in wave order.
constexpr int BFIN_ROWS = 64, BFIN_WAVES = 4;

__global__ __launch_bounds__(BFIN_ROWS * BFIN_WAVES) void k_band_finish(
    const float *__restrict__ recs, const int32_t *__restrict__ rec_start,
    const int32_t *__restrict__ rec_idx, int64_t n, const double *__restrict__ area,
    const double *__restrict__ x, double alpha, double beta, int trans, double scale1,
    double scale2, double *__restrict__ y)
{
    __shared__ double red[2][BFIN_WAVES][BFIN_ROWS];
    const int lane = threadIdx.x % BFIN_ROWS, w = threadIdx.x / BFIN_ROWS;
    const int64_t k = (int64_t)blockIdx.x * BFIN_ROWS + lane;
    double s1 = 0.0, s2 = 0.0;
    if (k < n) {
        const int K = (int)(k / TILE), l = (int)(k % TILE);
        for (int q = rec_start[K] + w; q < rec_start[K + 1]; q += BFIN_WAVES) {
            const float *r = recs + (int64_t)rec_idx[q] * (2 * TILE);
            s1 += (double)r[l];
            s2 += (double)r[TILE + l];
        }
    }
    red[0][w][lane] = s1;
    red[1][w][lane] = s2;
    __syncthreads();
    if (w != 0 || k >= n)
        return;
    s1 = red[0][0][lane];
    s2 = red[1][0][lane];
#pragma unroll
    for (int v = 1; v < BFIN_WAVES; ++v) {
        s1 += red[0][v][lane];
        s2 += red[1][v][lane];
    }
    if (trans) {
        const double sc = area[k] * INV_4PI;
        y[k] = alpha * x[k] - sc * scale2 * s2;
        y[n + k] = beta * x[n + k] - sc * scale1 * s1;
    } else {
        y[k] = alpha * x[k] - INV_4PI * scale1 * s1;
        y[n + k] = beta * x[n + k] - INV_4PI * scale2 * s2;
    }
}

// Row k = K*TILE + l: item rows of tile K, then the contributions of every tile
// I < K.  Blocks of 64 rows (one tile's worth of lanes, all in tile K); wave w
// of the 4 sums every 4th record of both lists, from record w on, and the four
// partial sums are added in wave order, so the result does not depend on
// scheduling.  Transposed, the two partial rows are output rows 2 and 1 and
// every row is scaled by its own area (and by scale1, scale2 as forward).
constexpr int FIN_ROWS = 64, FIN_WAVES = 4;

template <typename CT>
__global__ __launch_bounds__(FIN_ROWS * FIN_WAVES) void k_sym_finish(
    const double *__restrict__ rowpart, const CT *__restrict__ colpart,
    const int32_t *__restrict__ row_start, int T, int64_t n, const double *__restrict__ area,
    const double *__restrict__ x, double alpha, double beta, int trans, double scale1,
    double scale2, double *__restrict__ y)
{
    __shared__ double red[2][FIN_WAVES][FIN_ROWS];
    const int lane = threadIdx.x % FIN_ROWS, w = threadIdx.x / FIN_ROWS;
    const int64_t k = (int64_t)blockIdx.x * FIN_ROWS + lane;
    double s1 = 0.0, s2 = 0.0;
    if (k < n) {
        const int K = (int)(k / TILE), l = (int)(k % TILE);
        for (int q = row_start[K] + w; q < row_start[K + 1]; q += FIN_WAVES) {
            s1 += rowpart[(int64_t)q * (2 * TILE) + l];
            s2 += rowpart[(int64_t)q * (2 * TILE) + TILE + l];
        }
        for (int I = w; I < K; I += FIN_WAVES) {
            const CT *cp = colpart + sym_pair_index(I, K, T) * (2 * TILE);
            s1 += (double)cp[l];
            s2 += (double)cp[TILE + l];
        }
    }
    red[0][w][lane] = s1;
    red[1][w][lane] = s2;
    __syncthreads();
    if (w != 0 || k >= n)
        return;
    s1 = red[0][0][lane];
    s2 = red[1][0][lane];
#pragma unroll
    for (int v = 1; v < FIN_WAVES; ++v) {
        s1 += red[0][v][lane];
        s2 += red[1][v][lane];
    }
    if (trans) {
        const double sc = area[k] * INV_4PI;
        y[k] = alpha * x[k] - sc * scale2 * s2;
        y[n + k] = beta * x[n + k] - sc * scale1 * s1;
    } else {
        y[k] = alpha * x[k] - INV_4PI * scale1 * s1;
        y[n + k] = beta * x[n + k] - INV_4PI * scale2 * s2;
    }
}

// ---- pairwise FP64 sweep ----------------------------------------------------

// mode 0: w = a psi, f = a phi; mode 1 (transpose): w = l1, f = l2.
__global__ __launch_bounds__(TPB) void k_pack_sym64(const double *__restrict__ g, int64_t n,
                                                    int64_t npad, const double *__restrict__ x,
                                                    Src8d *__restrict__ src, int mode)
{
    const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (j >= npad)
        return;
    Src8d s;
    if (j < n) {
        const double a = g[6 * npad + j];
        const double w = mode ? x[j] : a * x[n + j];
        const double f = mode ? x[n + j] : a * x[j];
        s.x = g[j];
        s.y = g[npad + j];
        s.z = g[2 * npad + j];
        s.w = w;
        s.nx = g[3 * npad + j];
        s.ny = g[4 * npad + j];
        s.nz = g[5 * npad + j];
        s.f = f;
    } else {
        // padding: weightless points far away, 8 apart
        s.x = FAR_SRC + 8.0 * double(j - n);
        s.y = s.z = 0.0;
        s.w = s.f = s.nx = s.ny = s.nz = 0.0;
    }
    src[j] = s;
}

template <bool TRANS>
__global__ __launch_bounds__(SYM64_NT, SYM64_MIN_WAVES) void k_pairs_f64_sym(const Src8d *__restrict__ src,
                                                       const int4 *__restrict__ items, int T,
                                                       PairParams pp,
                                                       double *__restrict__ rowpart,
                                                       double *__restrict__ colpart)
{
    __shared__ Src8d sh[SYM64_NS];
    __shared__ double colw[SYM64_NT / 64][2 * SYM64_NS];
    __shared__ double acc[2 * SYM64_TT][SYM64_NT];
    const int4 it = items[blockIdx.x];   // (I, J0, J1, slot)
    sym_item_f64<TRANS>(src, it.x, it.y, it.z, T, Coef<double>(pp),
                        rowpart + (int64_t)it.w * (2 * TILE), colpart, sh, colw, acc);
}

__global__ __launch_bounds__(TPB) void k_matvec_finish(const double *__restrict__ part,
                                                       int n_chunks, int64_t npad, int64_t n,
                                                       const double *__restrict__ area,
                                                       const double *__restrict__ x,
                                                       double alpha, double beta, int trans,
                                                       double scale1, double scale2,
                                                       double *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    double s1 = 0.0, s2 = 0.0;
    for (int c = 0; c < n_chunks; ++c) {
        s1 += part[(int64_t)c * npad + i];
        s2 += part[(int64_t)(n_chunks + c) * npad + i];
    }
    const double sc = trans ? area[i] * INV_4PI : INV_4PI;
    y[i] = alpha * x[i] - sc * scale1 * s1;
    y[n + i] = beta * x[n + i] - sc * scale2 * s2;
}

// ---- source terms ----------------------------------------------------------

__global__ __launch_bounds__(TPB) void k_source(const double *__restrict__ g, int64_t n,
                                                int64_t npad, int64_t nc,
                                                const double *__restrict__ pos,
                                                const double *__restrict__ q, double scale,
                                                double *__restrict__ b)
{
    __shared__ double4 sh[TILE];
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const double xi = g[i], yi = g[npad + i], zi = g[2 * npad + i];
    const double nxi = g[3 * npad + i], nyi = g[4 * npad + i], nzi = g[5 * npad + i];
    double s1 = 0.0, s2 = 0.0;
    for (int64_t t0 = 0; t0 < nc; t0 += TILE) {
        __syncthreads();
        const int64_t k = t0 + threadIdx.x;
        sh[threadIdx.x] = (k < nc) ? make_double4(pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], q[k])
                                   : make_double4(FAR_SRC, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = (int)min((int64_t)TILE, nc - t0);
        for (int kk = 0; kk < cnt; ++kk) {
            const double4 c = sh[kk];
            const double dx = xi - c.x, dy = yi - c.y, dz = zi - c.z;
            const double ir = rsqrt_t(dx * dx + dy * dy + dz * dz);
            s1 += c.w * ir;
            s2 += c.w * (nxi * dx + nyi * dy + nzi * dz) * (ir * ir * ir);
        }
    }
    if (i < n) {
        b[i] = s1 * scale;      // S1 = (1/eps_in) sum q G0
        b[n + i] = -s2 * scale; // S2 = (1/eps_in) sum q nu_x.grad_x G0
    }
}

// ---- charge-target sweeps: reaction potential / solid angle -----------------

template <int MODE>
__global__ __launch_bounds__(TPB) void k_charge_pairs(const Src8<double> *__restrict__ src,
                                                      int64_t nc, const double *__restrict__ pos,
                                                      Sweep sw, PairParams pp,
                                                      double *__restrict__ part, int64_t ncpad)
{
    __shared__ Src8<double> sh[TILE];
    const int b = blockIdx.x;
    const int chunk = b % sw.n_chunks;
    const int tb = b / sw.n_chunks;
    const int64_t k = (int64_t)tb * TPB + threadIdx.x;
    const int64_t kk = k < nc ? k : nc - 1;
    const double yx = pos[3 * kk], yy = pos[3 * kk + 1], yz = pos[3 * kk + 2];
    const double eps = pp.eps, epsm1 = pp.eps - 1.0, kap = pp.kappa;
    Acc<double> acc;
    const int t0 = chunk * sw.tiles_per_chunk;
    const int t1 = min(sw.n_tiles, t0 + sw.tiles_per_chunk);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
        sh[threadIdx.x] = src[(int64_t)t * TILE + threadIdx.x];
        __syncthreads();
        double p = 0.0;
        for (int jj = 0; jj < TILE; ++jj) {
            const Src8<double> s = sh[jj];
            const double dx = yx - s.x, dy = yy - s.y, dz = yz - s.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsqrt_t(r2);
            const double u = ir * ir * ir;
            const double md = s.mx * dx + s.my * dy + s.mz * dz;
            if (MODE == 0) {
                const double kr = kap * (r2 * ir);
                const double e = exp_neg(kr);
                const double em1 = e - 1.0;
                const double tm1 = fma(kr, e, em1);
                const double g2 = fma(eps, tm1, epsm1);
                p = fma(-em1, ir * s.w, p);
                p = fma(g2 * md, u, p);
            } else {
                p = fma(-md, u, p);   // sum_j a_j n_j.(x_j - y) / r^3
            }
        }
        acc.add(p);
    }
    part[(int64_t)chunk * ncpad + k] = acc.value();
}

// Per-charge sums over the source chunks (one thread per charge), then
// out[0] = sum_k q_k per[k] in a fixed order by a single block.
__global__ __launch_bounds__(TPB) void k_charge_sum(const double *__restrict__ part,
                                                    int n_chunks, int64_t nc, int64_t ncpad,
                                                    double *__restrict__ per)
{
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k >= nc)
        return;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c)
        s += part[(int64_t)c * ncpad + k];
    per[k] = s;
}

__global__ __launch_bounds__(TPB) void k_weighted_total(const double *__restrict__ per,
                                                        const double *__restrict__ q, int64_t nc,
                                                        double scale, double *__restrict__ out)
{
    __shared__ double sh[TPB / 64];
    double tot = 0.0;
    for (int64_t k = threadIdx.x; k < nc; k += TPB)
        tot += q[k] * per[k];
    const double r = block_sum(tot, sh);
    if (threadIdx.x == 0)
        out[0] = scale * r;
}

// ---- adjoint (forces) --------------------------------------------------------
//
// E = (c_u/2) q^T B' xi with A xi = b(y) and B'_{k,.} = [a_j K2'(y_k,x_j) | a_j K1'(y_k,x_j)]
// (K' = 4 pi K).  The adjoint right-hand side w' = B'^T q, per triangle j
// (d = x_j - y_k, c_x = n_j.d):
//   w'1_j = -a_j sum_k q_k g2 c_x / r^3      (phi block, K2')
//   w'2_j = -a_j sum_k q_k (e - 1) / r       (psi block, K1')
__global__ __launch_bounds__(TPB) void k_adjoint_rhs(const double *__restrict__ g, int64_t n,
                                                     int64_t npad, int64_t nc,
                                                     const double *__restrict__ pos,
                                                     const double *__restrict__ q, double eps,
                                                     double kappa, double *__restrict__ w)
{
    __shared__ double4 sh[TILE];
    const int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const double xj = g[j], yj = g[npad + j], zj = g[2 * npad + j];
    const double nxj = g[3 * npad + j], nyj = g[4 * npad + j], nzj = g[5 * npad + j];
    const double epsm1 = eps - 1.0;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t t0 = 0; t0 < nc; t0 += TILE) {
        __syncthreads();
        const int64_t k = t0 + threadIdx.x;
        sh[threadIdx.x] = (k < nc) ? make_double4(pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], q[k])
                                   : make_double4(FAR_SRC, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = (int)min((int64_t)TILE, nc - t0);
        for (int kk = 0; kk < cnt; ++kk) {
            const double4 c = sh[kk];
            const double dx = xj - c.x, dy = yj - c.y, dz = zj - c.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsqrt_t(r2);
            const double kr = kappa * (r2 * ir);
            const double e = exp_neg(kr);
            const double em1 = e - 1.0;
            const double g2 = fma(eps, fma(kr, e, em1), epsm1);
            const double cxd = nxj * dx + nyj * dy + nzj * dz;
            s1 = fma(c.w * g2 * cxd, ir * ir * ir, s1);
            s2 = fma(c.w * em1, ir, s2);
        }
    }
    if (j < n) {
        const double a = g[6 * npad + j];
        w[j] = -a * s1;
        w[n + j] = -a * s2;
    }
}

// Per-charge sweep over triangles for the gradients (d = y_k - x_j):
//  out0: P'_k = sum_j [-(e-1)/r w_j + g2 (m_j.d) u]                (reaction potential)
//  out1-3: grad_y P'_k = sum_j u {d [w_j (kappa r e + e - 1) - eps kappa^2 e (m_j.d)
//                                    - 3 g2 (m_j.d)/r^2] + g2 m_j}
//  out4: c_k = sum_j [l_j / r + (p_j.d) u]                        (sum_i lam_i C'_ik eps_in)
//  out5-7: grad_y c_k = sum_j u [p_j - d (l_j + 3 (p_j.d)/r^2)]
// with (w, m) = (a psi, a phi n) from the forward stream and (l, p) =
// (lam1, lam2 n) from the transposed stream.
__global__ __launch_bounds__(TPB) void k_force_pairs(const Src8<double> *__restrict__ fwd,
                                                     const Src8<double> *__restrict__ adj,
                                                     int64_t nc, const double *__restrict__ pos,
                                                     Sweep sw, PairParams pp,
                                                     double *__restrict__ part, int64_t ncpad)
{
    __shared__ Src8<double> shf[TILE];
    __shared__ Src8<double> sha[TILE];
    const int b = blockIdx.x;
    const int chunk = b % sw.n_chunks;
    const int tb = b / sw.n_chunks;
    const int64_t k = (int64_t)tb * TPB + threadIdx.x;
    const int64_t kk = k < nc ? k : nc - 1;
    const double yx = pos[3 * kk], yy = pos[3 * kk + 1], yz = pos[3 * kk + 2];
    const double eps = pp.eps, epsm1 = pp.eps - 1.0, kap = pp.kappa, ek2 = pp.eps * kap * kap;
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int t0 = chunk * sw.tiles_per_chunk;
    const int t1 = min(sw.n_tiles, t0 + sw.tiles_per_chunk);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();
        shf[threadIdx.x] = fwd[(int64_t)t * TILE + threadIdx.x];
        sha[threadIdx.x] = adj[(int64_t)t * TILE + threadIdx.x];
        __syncthreads();
        for (int jj = 0; jj < TILE; ++jj) {
            const Src8<double> f = shf[jj];
            const Src8<double> a = sha[jj];
            const double dx = yx - f.x, dy = yy - f.y, dz = yz - f.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsqrt_t(r2);
            const double ir2 = ir * ir;
            const double u = ir2 * ir;
            const double kr = kap * (r2 * ir);
            const double e = exp_neg(kr);
            const double em1 = e - 1.0;
            const double g2 = fma(eps, fma(kr, e, em1), epsm1);
            const double md = f.mx * dx + f.my * dy + f.mz * dz;
            acc[0] = fma(-em1, ir * f.w, acc[0]);
            acc[0] = fma(g2 * md, u, acc[0]);
            const double cd = f.w * fma(kr, e, em1) - ek2 * e * md - 3.0 * g2 * md * ir2;
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
#pragma unroll
    for (int o = 0; o < 8; ++o)
        part[((int64_t)o * sw.n_chunks + chunk) * ncpad + k] = acc[o];
}

// dE/dq_k = (c_u/2) [P'_k + c_k/(4 pi eps_in)],
// dE/dy_k = (c_u/2) q_k [grad P'_k + grad c_k/(4 pi eps_in)]; per[k] = P'_k.
__global__ __launch_bounds__(TPB) void k_force_finish(const double *__restrict__ part,
                                                      int n_chunks, int64_t nc, int64_t ncpad,
                                                      const double *__restrict__ q,
                                                      double half_cu, double inv4pi_eps_in,
                                                      double *__restrict__ dpos,
                                                      double *__restrict__ dq,
                                                      double *__restrict__ per)
{
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k >= nc)
        return;
    double v[8];
    for (int o = 0; o < 8; ++o) {
        double s = 0.0;
        for (int c = 0; c < n_chunks; ++c)
            s += part[((int64_t)o * n_chunks + c) * ncpad + k];
        v[o] = s;
    }
    per[k] = v[0];
    dq[k] = half_cu * (v[0] + inv4pi_eps_in * v[4]);
    for (int d = 0; d < 3; ++d)
        dpos[3 * k + d] = half_cu * q[k] * (v[1 + d] + inv4pi_eps_in * v[5 + d]);
}

// ---- block-diagonal leaf preconditioner (Sec. 2.2.4) -------------------------
//
// One workgroup per leaf of m <= PC_MAX_LEAF elements: the 2m x 2m block of A
// on the leaf's indices (rows/columns [phi; psi] of the leaf) is assembled in
// LDS and inverted in place by Gauss-Jordan elimination with partial (row)
// pivoting; the inverse is stored column-major at inv + boff[leaf], so that
// the forward apply (every GMRES step) reads it along columns, consecutive
// rows in consecutive threads.  Applying M^-1 is then one small dense matvec
// per leaf.  The index table pq holds the
// phi and psi slots of the elements in leaf order.

__global__ __launch_bounds__(TPB) void k_pc_index(const int32_t *__restrict__ perm, int64_t n,
                                                  int64_t *__restrict__ pq)
{
    const int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n)
        return;
    pq[e] = perm[e];
    pq[n + e] = n + perm[e];
}

// One wave per leaf: lane i holds row i of the 2m x 2m block in registers
// (MM >= 2m columns, unrolled), the pivot of column k is the largest |A(i, k)|
// over rows not yet used (wave argmax, ties to the lower row), and only the
// scaled pivot row passes through LDS (a broadcast).  Rows are never moved:
// lane piv[k] ends with row k of the in-place inverse of the row-permuted
// block, so inverse(r, c) = A(piv[r], q[c]) with q the inverse permutation of
// piv.
constexpr int PC_LANES = 64;
constexpr int PC_SMALL_M2 = 64;   // largest block k_pc_build inverts in one wave

// Gauss-Jordan inversion of the 2m x 2m block held in LDS rows of stride LD
// (lane i: row i in registers, W >= 2m columns unrolled); writes the inverse
// column-major to out.
template <int W, int LD>
__device__ __forceinline__ void pc_invert(double *A, double *prow, int *piv, int *qinv, int m,
                                          double eps, double *__restrict__ out)
{
    const int lane = threadIdx.x, m2 = 2 * m;
    const bool mine = lane < m2;
    const double dg = lane < m ? 0.5 * (1.0 + eps) : 0.5 * (1.0 + 1.0 / eps);
    double row[W];   // every index below is a compile-time constant
#pragma unroll
    for (int c = 0; c < W; ++c)
        row[c] = (mine && c < m2) ? A[lane * LD + c] + (c == lane ? dg : 0.0) : 0.0;
    uint64_t used = 0;   // rows already chosen as pivots (the same in every lane)
    for (int k = 0; k < m2; ++k) {
        double ak = 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c)
            ak = (c == k) ? row[c] : ak;
        double v = (mine && !((used >> lane) & 1)) ? fabs(ak) : -1.0;
        int idx = lane;
#pragma unroll
        for (int off = PC_LANES / 2; off > 0; off >>= 1) {
            const double ov = __shfl_xor(v, off, PC_LANES);
            const int oi = __shfl_xor(idx, off, PC_LANES);
            if (ov > v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        const int p = idx;
        used |= 1ull << p;
        if (lane == p) {
            const double pinv = 1.0 / ak;
#pragma unroll
            for (int c = 0; c < W; ++c) {
                row[c] = (c == k) ? pinv : row[c] * pinv;
                prow[c] = row[c];
            }
            piv[k] = p;
        }
        __syncthreads();
        if (mine && lane != p) {
            const double pinv = prow[k];
#pragma unroll
            for (int c = 0; c < W; ++c)
                row[c] = (c == k) ? -ak * pinv : fma(-ak, prow[c], row[c]);
        }
        __syncthreads();
    }
    if (mine) {
#pragma unroll
        for (int c = 0; c < W; ++c)
            A[lane * LD + c] = row[c];
        qinv[piv[lane]] = lane;
    }
    __syncthreads();
    for (int e = lane; e < m2 * m2; e += PC_LANES) {
        const int c = e / m2, r = e - c * m2;
        out[e] = A[piv[r] * LD + qinv[c]];
    }
}

// The four entries -K_1..-K_4 (times a_q / 4 pi) that the leaf pair (r, q)
// contributes to the 2m x 2m block (rows/columns in leaf order, gp holds the
// leaf's centroids, normals and areas); all zero for r = q (j = i omitted).
// out[0]: (r, m + q), out[1]: (r, q), out[2]: (m + r, m + q), out[3]: (m + r, q).
template <int LMAX>
__device__ __forceinline__ void pc_pair(const double (*gp)[LMAX], int r, int q, double eps,
                                        double kappa, double (&out)[4])
{
    double k1 = 0.0, k2 = 0.0, k3 = 0.0, k4 = 0.0;
    if (r != q) {
        const double epsm1 = eps - 1.0, ieps = 1.0 / eps, iepsm1 = 1.0 / eps - 1.0;
        const double dx = gp[0][r] - gp[0][q], dy = gp[1][r] - gp[1][q];
        const double dz = gp[2][r] - gp[2][q];
        const double nxi = gp[3][r], nyi = gp[4][r], nzi = gp[5][r];
        const double nxj = gp[3][q], nyj = gp[4][q], nzj = gp[5][q];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ir = rsqrt_t(r2);
        const double ir2 = ir * ir, u = ir2 * ir;
        const double kr = kappa * (r2 * ir);
        const double ee = exp_neg(kr);
        const double em1 = ee - 1.0;
        const double tm1 = fma(kr, ee, em1);
        const double cx = nxi * dx + nyi * dy + nzi * dz;
        const double cy = nxj * dx + nyj * dy + nzj * dz;
        const double nn = nxi * nxj + nyi * nyj + nzi * nzj;
        const double h = fma(tm1, 3.0 * ir2, kappa * kappa * ee);
        k1 = -em1 * ir;
        k2 = fma(eps, tm1, epsm1) * cy * u;
        k3 = fma(ieps, tm1, iepsm1) * cx * u;
        k4 = u * (tm1 * nn - cx * cy * h);
    }
    const double aj = gp[6][q] * INV_4PI;
    out[0] = -k1 * aj;
    out[1] = -k2 * aj;
    out[2] = -k3 * aj;
    out[3] = -k4 * aj;
}

template <int MM>
__global__ __launch_bounds__(PC_LANES) void k_pc_build(const double *__restrict__ g,
                                                       int64_t npad,
                                                       const int32_t *__restrict__ perm,
                                                       const int32_t *__restrict__ lstart,
                                                       const int64_t *__restrict__ boff,
                                                       double eps, double kappa,
                                                       double *__restrict__ inv)
{
    __shared__ double A[MM][MM + 1];
    __shared__ double prow[MM];
    __shared__ double gp[7][MM / 2];   // the leaf's points: centroid, normal, area
    __shared__ int piv[MM], qinv[MM];
    const int l = blockIdx.x, lane = threadIdx.x;
    const int s0 = lstart[l];
    const int m = lstart[l + 1] - s0;
    const int m2 = 2 * m;
    if (m < 1 || m2 > MM)
        return;   // the host never builds such leaves; never overrun the LDS block
    if (lane < m) {
        const int64_t i = perm[s0 + lane];
#pragma unroll
        for (int k = 0; k < 7; ++k)
            gp[k][lane] = g[k * npad + i];
    }
    __syncthreads();
    for (int e = lane; e < m * m; e += PC_LANES) {
        const int r = e / m, q = e - r * m;   // rows and columns in leaf order
        double k[4];
        pc_pair<MM / 2>(gp, r, q, eps, kappa, k);
        A[r][q] = k[1];
        A[r][m + q] = k[0];
        A[m + r][q] = k[3];
        A[m + r][m + q] = k[2];
    }
    __syncthreads();
    double *out = inv + boff[l];
    // the unrolled width follows the leaf, not the bound
    if (m2 <= 16)
        pc_invert<16, MM + 1>(&A[0][0], prow, piv, qinv, m, eps, out);
    else if constexpr (MM >= 32) {
        if (m2 <= 32)
            pc_invert<32, MM + 1>(&A[0][0], prow, piv, qinv, m, eps, out);
        else if constexpr (MM >= 48) {
            if (m2 <= 48)
                pc_invert<48, MM + 1>(&A[0][0], prow, piv, qinv, m, eps, out);
            else if constexpr (MM >= 64)
                pc_invert<64, MM + 1>(&A[0][0], prow, piv, qinv, m, eps, out);
        }
    }
}

// Leaves with 64 < 2m <= 2 PC_MAX_LEAF: the block no longer fits one wave's
// registers (nor, in FP64, the LDS), so it is spread over the registers of a
// whole workgroup.  Thread t = 200 grp + c (t < 1000) owns the entries of
// column c in the rows r = grp + 5 j, j < 40, the same entries at every step
// (every register index is a compile-time constant but one, the pivot row's,
// which is uniform over the block).  Per column k: the five owners of column k
// publish it in LDS with their candidates for the pivot (largest |A(r, k)|
// over rows not yet used, ties to the lower row); the owners of the pivot row
// publish it scaled; every thread then updates its entries.  The pivoting
// rule and the read-out through the pivot permutation are those of pc_invert,
// so both kernels compute the same inverse up to rounding.
constexpr int PCB_COLS = 2 * PC_MAX_LEAF;            // 200
constexpr int PCB_GROUPS = 5;
constexpr int PCB_ROWS = PCB_COLS / PCB_GROUPS;       // 40 rows per thread
constexpr int PCB_THREADS = 1024;                     // 1000 working, 24 idle
static_assert(PCB_ROWS * PCB_GROUPS == PCB_COLS, "row groups must tile the block");

__global__ __launch_bounds__(PCB_THREADS) void k_pc_build_big(
    const double *__restrict__ g, int64_t npad, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ lstart, const int64_t *__restrict__ boff, double eps,
    double kappa, double *__restrict__ inv)
{
    __shared__ double gp[7][PC_MAX_LEAF];
    __shared__ double colk[PCB_COLS], prow[PCB_COLS];
    __shared__ double cv[PCB_GROUPS];
    __shared__ int ci[PCB_GROUPS];
    __shared__ int piv[PCB_COLS], qinv[PCB_COLS], used[PCB_COLS];
    const int l = blockIdx.x, t = threadIdx.x;
    const int s0 = lstart[l];
    const int m = lstart[l + 1] - s0;
    const int m2 = 2 * m;
    if (m2 <= PC_SMALL_M2 || m > PC_MAX_LEAF)
        return;   // small leaves are k_pc_build's; the test is uniform over the block
    const int c = t % PCB_COLS, grp = t / PCB_COLS;
    const bool active = grp < PCB_GROUPS && c < m2;
    for (int e = t; e < m; e += PCB_THREADS) {
        const int64_t i = perm[s0 + e];
#pragma unroll
        for (int k = 0; k < 7; ++k)
            gp[k][e] = g[k * npad + i];
    }
    for (int e = t; e < m2; e += PCB_THREADS)
        used[e] = 0;
    __syncthreads();
    const double alpha = 0.5 * (1.0 + eps), beta = 0.5 * (1.0 + 1.0 / eps);
    double a[PCB_ROWS];
#pragma unroll
    for (int j = 0; j < PCB_ROWS; ++j) {
        const int r = grp + PCB_GROUPS * j;
        double v = 0.0;
        if (active && r < m2) {
            double k[4];
            const int rr = r < m ? r : r - m, cc = c < m ? c : c - m;
            pc_pair<PC_MAX_LEAF>(gp, rr, cc, eps, kappa, k);
            // quadrant: (phi, psi) rows against (phi, psi) columns
            v = r < m ? (c < m ? k[1] : k[0]) : (c < m ? k[3] : k[2]);
            if (r == c)
                v += r < m ? alpha : beta;
        }
        a[j] = v;
    }
    for (int k = 0; k < m2; ++k) {
        if (active && c == k) {
            double best = -1.0;
            int bi = PCB_COLS;
#pragma unroll
            for (int j = 0; j < PCB_ROWS; ++j) {
                const int r = grp + PCB_GROUPS * j;
                if (r < m2) {
                    colk[r] = a[j];
                    const double v = used[r] ? -1.0 : fabs(a[j]);
                    if (v > best) {   // rows ascend with j: ties keep the lower row
                        best = v;
                        bi = r;
                    }
                }
            }
            cv[grp] = best;
            ci[grp] = bi;
        }
        __syncthreads();
        double bv = cv[0];
        int p = ci[0];
#pragma unroll
        for (int q = 1; q < PCB_GROUPS; ++q) {
            const double v = cv[q];
            const int i = ci[q];
            if (v > bv || (v == bv && i < p)) {
                bv = v;
                p = i;
            }
        }
        const double pinv = 1.0 / colk[p];
        if (active && grp == p % PCB_GROUPS) {
            const int jp = p / PCB_GROUPS;   // uniform over the block
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < PCB_ROWS; ++j)
                v = (j == jp) ? a[j] : v;
            prow[c] = (c == k) ? pinv : v * pinv;
            if (c == k) {
                used[p] = 1;
                piv[k] = p;
            }
        }
        __syncthreads();
        if (active) {
            const double pc = prow[c];
#pragma unroll
            for (int j = 0; j < PCB_ROWS; ++j) {
                const int r = grp + PCB_GROUPS * j;
                if (r < m2) {
                    if (r == p) {
                        a[j] = pc;
                    } else {
                        const double f = colk[r];
                        a[j] = (c == k) ? -f * pinv : fma(-f, pc, a[j]);
                    }
                }
            }
        }
        __syncthreads();
    }
    for (int k = t; k < m2; k += PCB_THREADS)
        qinv[piv[k]] = k;
    __syncthreads();
    if (active) {
        double *out = inv + boff[l];
        const int pc = piv[c];
#pragma unroll
        for (int j = 0; j < PCB_ROWS; ++j) {
            const int r = grp + PCB_GROUPS * j;
            if (r < m2)
                out[(int64_t)pc * m2 + qinv[r]] = a[j];   // column-major
        }
    }
}

// y = M^-1 x (or M^-T x): one workgroup per leaf.  pidx/qidx give the
// vector positions of the phi and psi unknowns of the leaf's elements.
__global__ __launch_bounds__(TPB) void k_pc_apply(const double *__restrict__ inv,
                                                  const int64_t *__restrict__ boff,
                                                  const int64_t *__restrict__ pidx,
                                                  const int64_t *__restrict__ qidx,
                                                  const int32_t *__restrict__ lstart,
                                                  const double *__restrict__ x, int trans,
                                                  double *__restrict__ y)
{
    constexpr int MM = 2 * PC_MAX_LEAF;
    __shared__ double v[MM];
    const int l = blockIdx.x;
    const int s0 = lstart[l];
    const int m = lstart[l + 1] - s0;
    const int m2 = 2 * m;
    if (m < 1 || m > PC_MAX_LEAF)
        return;
    for (int r = threadIdx.x; r < m2; r += TPB)
        v[r] = (r < m) ? x[pidx[s0 + r]] : x[qidx[s0 + r - m]];
    __syncthreads();
    const double *B = inv + boff[l];   // column-major: B(r, c) = B[c m2 + r]
    // a thread per row; forward reads down the columns (consecutive rows in
    // consecutive threads), transposed along the rows
    for (int r = threadIdx.x; r < m2; r += TPB) {
        double s = 0.0;
        if (!trans) {
            for (int c = 0; c < m2; ++c)
                s = fma(B[(int64_t)c * m2 + r], v[c], s);
        } else {
            for (int c = 0; c < m2; ++c)
                s = fma(B[(int64_t)r * m2 + c], v[c], s);
        }
        if (r < m)
            y[pidx[s0 + r]] = s;
        else
            y[qidx[s0 + r - m]] = s;
    }
}

// ---- the FP64 pair functions, evaluated one argument per thread -------------
// exp(-x) and 1/sqrt(y) exactly as the FP64 pair sweeps compute them
// (pb_eval_pair_math).
__global__ __launch_bounds__(TPB) void k_eval_pair_math(int64_t n, const double *__restrict__ x,
                                                        const double *__restrict__ y,
                                                        double *__restrict__ ex,
                                                        double *__restrict__ rq)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n) {
        ex[i] = dev::exp_neg_pair(x[i]);
        rq[i] = dev::rsqrt_pos(y[i]);
    }
}

// ---- counter-calibration probe ------------------------------------------------
// Each thread runs PROBE_CH independent chains of PROBE_ITER steps of one
// operation, so the count of that operation is known exactly:
// KIND 0: x = fma(x, a, b) in FP32; 1: the same in FP64; 2: x = fma(exp2(x),
// a, b) in FP32 (one hardware exp2, a transcendental, and one FMA per step;
// with a = 1/2, b = 0 the chain stays at x = 1).  The chains are summed and
// stored so that nothing is dropped as dead code.
constexpr int PROBE_CH = 8, PROBE_ITER = 1024;

template <int KIND>
__global__ __launch_bounds__(TPB) void k_probe_valu(float a, float b, double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if constexpr (KIND == 1) {
        double x[PROBE_CH];
#pragma unroll
        for (int c = 0; c < PROBE_CH; ++c)
            x[c] = 1.0 + (double)c * 0.125;
        for (int it = 0; it < PROBE_ITER; ++it) {
#pragma unroll
            for (int c = 0; c < PROBE_CH; ++c)
                x[c] = fma(x[c], (double)a, (double)b);
        }
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < PROBE_CH; ++c)
            sum += x[c];
        out[t] = sum;
    } else {
        float x[PROBE_CH];
#pragma unroll
        for (int c = 0; c < PROBE_CH; ++c)
            x[c] = 1.0f + (float)c * 0.125f;
        for (int it = 0; it < PROBE_ITER; ++it) {
#pragma unroll
            for (int c = 0; c < PROBE_CH; ++c) {
                if constexpr (KIND == 0)
                    x[c] = fmaf(x[c], a, b);
                else
                    x[c] = fmaf(__builtin_amdgcn_exp2f(x[c]), a, b);
            }
        }
        float sum = 0.f;
#pragma unroll
        for (int c = 0; c < PROBE_CH; ++c)
            sum += x[c];
        out[t] = (double)sum;
    }
}

// ---- Coulomb potential of the charges at arbitrary points --------------------
// out_k = scale * sum_l q_l / |x_k - y_l|, l == k skipped when skip_self
// (x = the charges themselves).
__global__ __launch_bounds__(TPB) void k_point_coulomb(int64_t npts, const double *__restrict__ pts,
                                                       int64_t nc, const double *__restrict__ pos,
                                                       const double *__restrict__ q, double scale,
                                                       int skip_self, double *__restrict__ out)
{
    __shared__ double4 sh[TILE];
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t kk = k < npts ? k : npts - 1;
    const double x = pts[3 * kk], y = pts[3 * kk + 1], z = pts[3 * kk + 2];
    double s = 0.0;
    for (int64_t t0 = 0; t0 < nc; t0 += TILE) {
        __syncthreads();
        const int64_t l = t0 + threadIdx.x;
        sh[threadIdx.x] = (l < nc) ? make_double4(pos[3 * l], pos[3 * l + 1], pos[3 * l + 2], q[l])
                                   : make_double4(FAR_SRC, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = (int)min((int64_t)TILE, nc - t0);
        for (int ll = 0; ll < cnt; ++ll) {
            if (skip_self && t0 + ll == k)
                continue;
            const double4 c = sh[ll];
            const double dx = x - c.x, dy = y - c.y, dz = z - c.z;
            s += c.w * rsqrt_t(dx * dx + dy * dy + dz * dz);
        }
    }
    if (k < npts)
        out[k] = scale * s;
}

// ---- BLAS-1 ----------------------------------------------------------------

__global__ __launch_bounds__(TPB) void k_dots(const double *__restrict__ V, int64_t ld, int k,
                                              const double *__restrict__ w, int64_t n,
                                              double *__restrict__ part, int nblk)
{
    __shared__ double sh[TPB / 64];
    const int j = blockIdx.y;
    const double *a = (j < k) ? V + (int64_t)j * ld : w;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)nblk * TPB)
        s = fma(a[i], w[i], s);
    const double r = block_sum(s, sh);
    if (threadIdx.x == 0)
        part[(int64_t)j * nblk + blockIdx.x] = r;
}

__global__ __launch_bounds__(TPB) void k_reduce_cols(const double *__restrict__ part, int nblk,
                                                     double *__restrict__ out)
{
    __shared__ double sh[TPB / 64];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += TPB)
        s += part[(int64_t)j * nblk + b];
    const double r = block_sum(s, sh);
    if (threadIdx.x == 0)
        out[j] = r;
}

__global__ __launch_bounds__(TPB) void k_sub_basis(const double *__restrict__ V, int64_t ld,
                                                   int k, const double *__restrict__ h,
                                                   double *__restrict__ w, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    double s = w[i];
    for (int j = 0; j < k; ++j)
        s -= h[j] * V[(int64_t)j * ld + i];
    w[i] = s;
}

__global__ __launch_bounds__(TPB) void k_scale_inv_sqrt(const double *__restrict__ w,
                                                        const double *__restrict__ nrm2,
                                                        double *__restrict__ v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const double s2 = nrm2[0];
    v[i] = (s2 > 0.0) ? w[i] / sqrt(s2) : 0.0;
}

__global__ __launch_bounds__(TPB) void k_add_basis(const double *__restrict__ V, int64_t ld,
                                                   int k, const double *__restrict__ y,
                                                   double *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    double s = 0.0;
    for (int j = 0; j < k; ++j)
        s += y[j] * V[(int64_t)j * ld + i];
    x[i] += s;
}

__global__ __launch_bounds__(TPB) void k_sub(const double *__restrict__ b,
                                             const double *__restrict__ ax,
                                             double *__restrict__ r, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n)
        r[i] = b[i] - ax[i];
}

__global__ __launch_bounds__(TPB) void k_add(double *__restrict__ x, const double *__restrict__ d,
                                             int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n)
        x[i] += d[i];
}

__global__ __launch_bounds__(TPB) void k_fill(double *__restrict__ x, double v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n)
        x[i] = v;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

// ---- host-side launchers ------------------------------------------------------

Sweep plan_sweep(int64_t n_targets, int64_t n_sources, int target_waves, int tpt)
{
    Sweep s;
    const int64_t per_block = (int64_t)TPB * tpt;
    s.n_tblocks = (int)((n_targets + per_block - 1) / per_block);
    s.n_tiles = (int)((n_sources + TILE - 1) / TILE);
    if (s.n_tiles < 1)
        s.n_tiles = 1;
    const int waves_per_chunk = s.n_tblocks * (TPB / 64);
    int want = (target_waves + waves_per_chunk - 1) / waves_per_chunk;
    if (want >= 8)
        want = (want + 7) / 8 * 8;   // whole XCD rounds
    if (want > s.n_tiles)
        want = s.n_tiles;
    if (want < 1)
        want = 1;
    s.tiles_per_chunk = (s.n_tiles + want - 1) / want;
    s.n_chunks = (s.n_tiles + s.tiles_per_chunk - 1) / s.tiles_per_chunk;
    return s;
}

void launch_dup_check(hipStream_t s, const double *g, int64_t n, int64_t ld, int32_t *tab,
                      int64_t cap)
{
    const unsigned cb = (unsigned)std::min<int64_t>((cap + 2 + TPB - 1) / TPB, 4096);
    hipLaunchKernelGGL(k_dup_clear, dim3(cb), dim3(TPB), 0, s, tab, cap);
    hipLaunchKernelGGL(k_dup_insert, dim3(blocks_for(n)), dim3(TPB), 0, s, g, n, ld, tab, cap);
}

int geometry_blocks(int64_t n_tri)
{
    int64_t b = (n_tri + TPB - 1) / TPB;
    if (b > 1024)
        b = 1024;
    if (b < 1)
        b = 1;
    return (int)b;
}

void launch_geometry(hipStream_t s, int64_t n_vert, int64_t n_tri, const double *vert,
                     const int32_t *tri, double *g, int64_t npad, int64_t ld, double *part,
                     int nblk)
{
    hipLaunchKernelGGL(k_geometry, dim3(nblk), dim3(TPB), 0, s, n_vert, n_tri, vert, tri, g, npad,
                       ld, part, nblk);
}

void launch_pack_f64(hipStream_t s, const Geo &geo, const double *x, double *src, int mode)
{
    hipLaunchKernelGGL(k_pack<double>, dim3(blocks_for(geo.npad)), dim3(TPB), 0, s, geo.g, geo.n,
                       geo.npad, x, reinterpret_cast<Src8<double> *>(src), mode, 0.0, 0.0, 0.0,
                       1.0, 1.0);
}

void launch_pack_f32(hipStream_t s, const Geo &geo, const double *x, float *src, int mode,
                     double cx, double cy, double cz, double eps, double sigma)
{
    hipLaunchKernelGGL(k_pack<float>, dim3(blocks_for(geo.npad)), dim3(TPB), 0, s, geo.g, geo.n,
                       geo.npad, x, reinterpret_cast<Src8<float> *>(src), mode, cx, cy, cz, eps,
                       sigma);
}

void launch_pairs_f32_fwd(hipStream_t s, const Geo &geo, const float *src, const Sweep &sw,
                          const PairParams &pp, int tpt, double *part)
{
    const dim3 grid(sw.n_tblocks * sw.n_chunks);
    const auto *p = reinterpret_cast<const Src8<float> *>(src);
    const bool scaled = f32_scaled(pp);
    if (tpt == 2 && scaled)
        hipLaunchKernelGGL((k_pairs_f32_fwd<2, true>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad,
                           sw, pp, part);
    else if (tpt == 2)
        hipLaunchKernelGGL((k_pairs_f32_fwd<2, false>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad,
                           sw, pp, part);
    else if (scaled)
        hipLaunchKernelGGL((k_pairs_f32_fwd<1, true>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad,
                           sw, pp, part);
    else
        hipLaunchKernelGGL((k_pairs_f32_fwd<1, false>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad,
                           sw, pp, part);
}

void launch_pack_sym(hipStream_t s, const Geo &geo, const double *x, float *src, double cx,
                     double cy, double cz, double eps, double sigma, int mode)
{
    hipLaunchKernelGGL(k_pack_sym, dim3(blocks_for(geo.npad)), dim3(TPB), 0, s, geo.g, geo.n,
                       geo.npad, x, reinterpret_cast<Src12 *>(src), cx, cy, cz, eps, sigma, mode);
}

void launch_pairs_f32_sym(hipStream_t s, const float *src, const int32_t *items, int n_items,
                          int n_tiles, const PairParams &pp, int transpose, double *rowpart,
                          float *colpart)
{
    const auto *p = reinterpret_cast<const Src12 *>(src);
    const auto *it = reinterpret_cast<const int4 *>(items);
    PairParams q = pp;
    if (transpose)
        q.eps = 1.0 / pp.eps;   // the pair constant of the transposed reduced form
    if (f32_scaled(q))
        hipLaunchKernelGGL(k_pairs_f32_sym<true>, dim3(n_items), dim3(SYM_NT), 0, s, p, it,
                           n_tiles, q, rowpart, colpart);
    else
        hipLaunchKernelGGL(k_pairs_f32_sym<false>, dim3(n_items), dim3(SYM_NT), 0, s, p, it,
                           n_tiles, q, rowpart, colpart);
}

void launch_sym_finish(hipStream_t s, const Geo &geo, const double *rowpart,
                       const float *colpart, const int32_t *row_start, int n_tiles,
                       const double *x, double alpha, double beta, int transpose, double scale1,
                       double scale2, double *y)
{
    hipLaunchKernelGGL(k_sym_finish<float>, dim3((geo.n + FIN_ROWS - 1) / FIN_ROWS),
                       dim3(FIN_ROWS * FIN_WAVES), 0, s, rowpart,
                       colpart, row_start, n_tiles, geo.n, geo.g + 6 * geo.npad, x,
                       alpha, beta, transpose, scale1, scale2, y);
}

void launch_pairs_f32_band(hipStream_t s, const float *src, const BandItem *items, int n_items,
                           int n_tiles, const PairParams &pp, int transpose, float *recs)
{
    const auto *p = reinterpret_cast<const Src12 *>(src);
    PairParams q = pp;
    if (transpose)
        q.eps = 1.0 / pp.eps;   // the pair constant of the transposed reduced form
    if (f32_scaled(q))
        hipLaunchKernelGGL(k_pairs_f32_band<true>, dim3(n_items), dim3(BAND_WAVES * 64), 0, s, p,
                           items, n_tiles, q, recs);
    else
        hipLaunchKernelGGL(k_pairs_f32_band<false>, dim3(n_items), dim3(BAND_WAVES * 64), 0, s,
                           p, items, n_tiles, q, recs);
}

void launch_band_finish(hipStream_t s, const Geo &geo, const float *recs,
                        const int32_t *rec_start, const int32_t *rec_idx, const double *x,
                        double alpha, double beta, int transpose, double scale1, double scale2,
                        double *y)
{
    hipLaunchKernelGGL(k_band_finish, dim3((geo.n + BFIN_ROWS - 1) / BFIN_ROWS),
                       dim3(BFIN_ROWS * BFIN_WAVES), 0, s, recs, rec_start, rec_idx, geo.n,
                       geo.g + 6 * geo.npad, x, alpha, beta, transpose, scale1, scale2, y);
}

void launch_pack_sym64(hipStream_t s, const Geo &geo, const double *x, double *src, int mode)
{
    hipLaunchKernelGGL(k_pack_sym64, dim3(blocks_for(geo.npad)), dim3(TPB), 0, s, geo.g, geo.n,
                       geo.npad, x, reinterpret_cast<Src8d *>(src), mode);
}

void launch_pairs_f64_sym(hipStream_t s, const double *src, const int32_t *items, int n_items,
                          int n_tiles, const PairParams &pp, int transpose, double *rowpart,
                          double *colpart)
{
    const auto *p = reinterpret_cast<const Src8d *>(src);
    const auto *it = reinterpret_cast<const int4 *>(items);
    if (transpose)
        hipLaunchKernelGGL(k_pairs_f64_sym<true>, dim3(n_items), dim3(SYM64_NT), 0, s, p, it, n_tiles,
                           pp, rowpart, colpart);
    else
        hipLaunchKernelGGL(k_pairs_f64_sym<false>, dim3(n_items), dim3(SYM64_NT), 0, s, p, it, n_tiles,
                           pp, rowpart, colpart);
}

void launch_sym_finish64(hipStream_t s, const Geo &geo, const double *rowpart,
                         const double *colpart, const int32_t *row_start, int n_tiles,
                         const double *x, double alpha, double beta, int transpose, double *y)
{
    hipLaunchKernelGGL(k_sym_finish<double>, dim3((geo.n + FIN_ROWS - 1) / FIN_ROWS),
                       dim3(FIN_ROWS * FIN_WAVES), 0, s, rowpart,
                       colpart, row_start, n_tiles, geo.n, geo.g + 6 * geo.npad, x,
                       alpha, beta, transpose, 1.0, 1.0, y);
}

void launch_pairs_f64(hipStream_t s, const Geo &geo, const double *src, const Sweep &sw,
                      const PairParams &pp, int transpose, double *part)
{
    const dim3 grid(sw.n_tblocks * sw.n_chunks);
    const auto *p = reinterpret_cast<const Src8<double> *>(src);
    PairParams q = pp;
    q.cx = q.cy = q.cz = 0.0;   // FP64 works in the caller's frame
    if (transpose)
        hipLaunchKernelGGL((k_pairs<double, true>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad, sw,
                           q, part);
    else
        hipLaunchKernelGGL((k_pairs<double, false>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad, sw,
                           q, part);
}

void launch_pairs_f32(hipStream_t s, const Geo &geo, const float *src, const Sweep &sw,
                      const PairParams &pp, int transpose, double *part)
{
    const dim3 grid(sw.n_tblocks * sw.n_chunks);
    const auto *p = reinterpret_cast<const Src8<float> *>(src);
    if (transpose)
        hipLaunchKernelGGL((k_pairs<float, true>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad, sw,
                           pp, part);
    else
        hipLaunchKernelGGL((k_pairs<float, false>), grid, dim3(TPB), 0, s, p, geo.g, geo.npad, sw,
                           pp, part);
}

void launch_matvec_finish(hipStream_t s, const Geo &geo, const double *part, int n_chunks,
                          const double *x, double alpha, double beta, int transpose,
                          double scale1, double scale2, double *y)
{
    hipLaunchKernelGGL(k_matvec_finish, dim3(blocks_for(geo.n)), dim3(TPB), 0, s, part, n_chunks,
                       geo.npad, geo.n, geo.g + 6 * geo.npad, x, alpha, beta, transpose, scale1,
                       scale2, y);
}

void launch_source(hipStream_t s, const Geo &geo, int64_t nc, const double *pos,
                   const double *q, double eps_in, double *b)
{
    hipLaunchKernelGGL(k_source, dim3(blocks_for(geo.npad)), dim3(TPB), 0, s, geo.g, geo.n,
                       geo.npad, nc, pos, q, INV_4PI / eps_in, b);
}

void launch_charge_pairs(hipStream_t s, const Geo &geo, const double *src, int64_t nc,
                         const double *pos, const Sweep &sw, const PairParams &pp, int mode,
                         double *part, int64_t ncpad)
{
    (void)geo;
    const dim3 grid(sw.n_tblocks * sw.n_chunks);
    const auto *p = reinterpret_cast<const Src8<double> *>(src);
    if (mode == 0)
        hipLaunchKernelGGL(k_charge_pairs<0>, grid, dim3(TPB), 0, s, p, nc, pos, sw, pp, part,
                           ncpad);
    else
        hipLaunchKernelGGL(k_charge_pairs<1>, grid, dim3(TPB), 0, s, p, nc, pos, sw, pp, part,
                           ncpad);
}

void launch_charge_finish(hipStream_t s, const double *part, int n_chunks, int64_t nc,
                          int64_t ncpad, const double *q, double scale, double *per, double *out)
{
    hipLaunchKernelGGL(k_charge_sum, dim3(blocks_for(nc)), dim3(TPB), 0, s, part, n_chunks, nc,
                       ncpad, per);
    if (q && out)
        hipLaunchKernelGGL(k_weighted_total, dim3(1), dim3(TPB), 0, s, per, q, nc, scale, out);
}

void launch_adjoint_rhs(hipStream_t s, const Geo &geo, int64_t nc, const double *pos,
                        const double *q, double eps, double kappa, double *w)
{
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(blocks_for(geo.npad)), dim3(TPB), 0, s, geo.g, geo.n,
                       geo.npad, nc, pos, q, eps, kappa, w);
}

void launch_force_pairs(hipStream_t s, const double *fwd, const double *adj, int64_t nc,
                        const double *pos, const Sweep &sw, const PairParams &pp, double *part,
                        int64_t ncpad)
{
    hipLaunchKernelGGL(k_force_pairs, dim3(sw.n_tblocks * sw.n_chunks), dim3(TPB), 0, s,
                       reinterpret_cast<const Src8<double> *>(fwd),
                       reinterpret_cast<const Src8<double> *>(adj), nc, pos, sw, pp, part, ncpad);
}

void launch_force_finish(hipStream_t s, const double *part, int n_chunks, int64_t nc,
                         int64_t ncpad, const double *q, double half_cu, double inv4pi_eps_in,
                         double *dpos, double *dq, double *per, double *out)
{
    hipLaunchKernelGGL(k_force_finish, dim3(blocks_for(nc)), dim3(TPB), 0, s, part, n_chunks, nc,
                       ncpad, q, half_cu, inv4pi_eps_in, dpos, dq, per);
    hipLaunchKernelGGL(k_weighted_total, dim3(1), dim3(TPB), 0, s, per, q, nc, half_cu, out);
}

void launch_pc_index(hipStream_t s, const int32_t *perm, int64_t n, int64_t *pq)
{
    hipLaunchKernelGGL(k_pc_index, dim3(blocks_for(n)), dim3(TPB), 0, s, perm, n, pq);
}

void launch_pc_build(hipStream_t s, const Geo &geo, const int32_t *perm, const int32_t *lstart,
                     const int64_t *boff, int64_t n_leaves, int max_leaf, double eps,
                     double kappa, double *inv)
{
    const int mm = std::min(2 * std::min(std::max(max_leaf, 1), PC_MAX_LEAF), PC_SMALL_M2);
    const dim3 grid((unsigned)n_leaves), block(PC_LANES);
    if (2 * max_leaf > PC_SMALL_M2)   // leaves of more than 32 elements, if any
        hipLaunchKernelGGL(k_pc_build_big, grid, dim3(PCB_THREADS), 0, s, geo.g, geo.npad, perm,
                           lstart, boff, eps, kappa, inv);
    if (mm <= 16)
        hipLaunchKernelGGL(k_pc_build<16>, grid, block, 0, s, geo.g, geo.npad, perm, lstart,
                           boff, eps, kappa, inv);
    else if (mm <= 32)
        hipLaunchKernelGGL(k_pc_build<32>, grid, block, 0, s, geo.g, geo.npad, perm, lstart,
                           boff, eps, kappa, inv);
    else if (mm <= 48)
        hipLaunchKernelGGL(k_pc_build<48>, grid, block, 0, s, geo.g, geo.npad, perm, lstart,
                           boff, eps, kappa, inv);
    else
        hipLaunchKernelGGL(k_pc_build<64>, grid, block, 0, s, geo.g, geo.npad, perm, lstart,
                           boff, eps, kappa, inv);
}

void launch_pc_apply(hipStream_t s, const double *inv, const int64_t *boff, const int64_t *pidx,
                     const int64_t *qidx, const int32_t *lstart, int64_t n_leaves,
                     const double *x, int trans, double *y)
{
    hipLaunchKernelGGL(k_pc_apply, dim3((unsigned)n_leaves), dim3(TPB), 0, s, inv, boff, pidx,
                       qidx, lstart, x, trans, y);
}

void launch_eval_pair_math(hipStream_t s, int64_t n, const double *x, const double *y,
                           double *ex, double *rq)
{
    hipLaunchKernelGGL(k_eval_pair_math, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s,
                       n, x, y, ex, rq);
}

int64_t launch_probe_valu(hipStream_t s, int kind, double *out)
{
    const dim3 grid((unsigned)(PROBE_THREADS / TPB)), block(TPB);
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_valu<0>, grid, block, 0, s, 0.999f, 1e-3f, out);
    else if (kind == 1)
        hipLaunchKernelGGL(k_probe_valu<1>, grid, block, 0, s, 0.999f, 1e-3f, out);
    else
        hipLaunchKernelGGL(k_probe_valu<2>, grid, block, 0, s, 0.5f, 0.0f, out);
    return PROBE_THREADS * PROBE_CH * PROBE_ITER;
}

void launch_point_coulomb(hipStream_t s, int64_t npts, const double *pts, int64_t nc,
                          const double *pos, const double *q, double scale, int skip_self,
                          double *out)
{
    hipLaunchKernelGGL(k_point_coulomb, dim3(blocks_for(npts)), dim3(TPB), 0, s, npts, pts, nc, pos,
                       q, scale, skip_self, out);
}

void launch_weighted_total(hipStream_t s, const double *per, const double *q, int64_t nc,
                           double scale, double *out)
{
    hipLaunchKernelGGL(k_weighted_total, dim3(1), dim3(TPB), 0, s, per, q, nc, scale, out);
}

int dot_blocks(int64_t n)
{
    int64_t b = (n + TPB - 1) / TPB;
    if (b > 512)
        b = 512;
    if (b < 1)
        b = 1;
    return (int)b;
}

void launch_dots(hipStream_t s, const double *V, int64_t ld, int k, const double *w, int64_t n,
                 double *part, int nblk)
{
    hipLaunchKernelGGL(k_dots, dim3(nblk, k + 1), dim3(TPB), 0, s, V, ld, k, w, n, part, nblk);
}

void launch_reduce_cols(hipStream_t s, const double *part, int nblk, int ncol, double *out)
{
    hipLaunchKernelGGL(k_reduce_cols, dim3(ncol), dim3(TPB), 0, s, part, nblk, out);
}

void launch_sub_basis(hipStream_t s, const double *V, int64_t ld, int k, const double *h,
                      double *w, int64_t n)
{
    hipLaunchKernelGGL(k_sub_basis, dim3(blocks_for(n)), dim3(TPB), 0, s, V, ld, k, h, w, n);
}

void launch_scale_inv_sqrt(hipStream_t s, const double *w, const double *nrm2, double *v,
                           int64_t n)
{
    hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(blocks_for(n)), dim3(TPB), 0, s, w, nrm2, v, n);
}

void launch_add_basis(hipStream_t s, const double *V, int64_t ld, int k, const double *y,
                      double *x, int64_t n)
{
    hipLaunchKernelGGL(k_add_basis, dim3(blocks_for(n)), dim3(TPB), 0, s, V, ld, k, y, x, n);
}

void launch_sub(hipStream_t s, const double *b, const double *ax, double *r, int64_t n)
{
    hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(TPB), 0, s, b, ax, r, n);
}

void launch_add(hipStream_t s, double *x, const double *d, int64_t n)
{
    hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(TPB), 0, s, x, d, n);
}

void launch_fill(hipStream_t s, double *x, double v, int64_t n)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(TPB), 0, s, x, v, n);
}

}  // namespace pbk
