// Treecode matvec (Sec. 2.2.3): the pair sums of the discretized
// eqs. eqbim_5/6 split into particle-particle sums over near leaves and
// p-th order Cartesian Taylor approximations for clusters that satisfy the
// multipole acceptance criterion r_c / R <= theta.
//
// Tree: the octree of the collocation points (root = the bounding box's
// centre and half its largest extent; a cluster with more than N0 points is
// split into its non-empty octants (x >= c) + 2 (y >= c) + 4 (z >= c)).  It is
// stored in depth-first order, so every cluster's points are one contiguous
// range of the permuted order and its subtree ends at `next`: a walk needs no
// stack.  Each cluster carries the centre of the tight bounding box of its
// points and half that box's diagonal as r_c.
//
// Expansion: each kernel K1..K4 is replaced by its p-th order Taylor
// polynomial in the source position about the cluster centre x_c.  With T^m
// the coefficients of F(x - x_c - h) in h (F = G0 = 1/r or G_kappa =
// exp(-kappa r)/r), the cluster moments are M^k = sum_j a_j psi_j h_j^k and
// D_d^k = sum_j a_j phi_j n_jd h_j^k (|k| <= p); a source normal derivative
// turns T^k into (k_d + 1) T^(k + e_d), a target normal derivative turns T^m
// into -(m_e + 1) T^(m + e_e), so coefficients to order p + 2 are needed.
// They come from the recurrences of the Cartesian treecode for screened
// Coulomb interactions (Li, Johnston and Krasny): for |k| = n >= 1,
//   n rho^2 a_k = (2n - 1) sum_i R_i a_(k - e_i) - (n - 1) sum_i a_(k - 2 e_i)
//                 + kappa (sum_i R_i b_(k - e_i) - sum_i b_(k - 2 e_i)),
//   n b_k = kappa (sum_i R_i a_(k - e_i) - sum_i a_(k - 2 e_i)),
// with a_0 = exp(-kappa rho)/rho and b_0 = exp(-kappa rho) (kappa = 0 gives
// the Coulomb coefficients).  All arithmetic is FP64.
#include "pb_ctx.h"
#include "pb_device.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace pbk {

namespace {

using namespace dev;

// number of multi-indices with |k| <= P
__host__ __device__ constexpr int nterms(int P) { return (P + 1) * (P + 2) * (P + 3) / 6; }

// position of k in graded order: |k| ascending, then k1 descending, then k2
// descending
__host__ __device__ constexpr int mi(int k1, int k2, int k3)
{
    return nterms(k1 + k2 + k3 - 1) + (k2 + k3) * (k2 + k3 + 1) / 2 + k3;
}

struct TreeNode {
    int lo, hi, next, leaf;
};

// ---- per-matvec kernels -----------------------------------------------------

// Permuted weights: w = a psi, v = a phi in tree order.
__global__ __launch_bounds__(TPB) void kt_gather(const int32_t *__restrict__ perm, int64_t n,
                                                 const double *__restrict__ area,
                                                 const double *__restrict__ x,
                                                 double *__restrict__ wv)
{
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k >= n)
        return;
    const int32_t i = perm[k];
    wv[k] = area[i] * x[n + i];
    wv[n + k] = area[i] * x[i];
}

// Moments of one cluster per block: M^k, then D_1^k, D_2^k, D_3^k.
template <int P>
__global__ __launch_bounds__(TPB) void kt_moments(const TreeNode *__restrict__ nodes,
                                                  const double4 *__restrict__ ctr,
                                                  const double *__restrict__ tg, int64_t n,
                                                  const double *__restrict__ wv,
                                                  double *__restrict__ mom)
{
    constexpr int NT = nterms(P);
    __shared__ double red[TPB / 64][4 * NT];
    const TreeNode nd = nodes[blockIdx.x];
    const double4 c = ctr[blockIdx.x];
    double acc[4 * NT];
#pragma unroll
    for (int t = 0; t < 4 * NT; ++t)
        acc[t] = 0.0;
    for (int k = nd.lo + (int)threadIdx.x; k < nd.hi; k += TPB) {
        const double h[3] = {tg[k] - c.x, tg[n + k] - c.y, tg[2 * n + k] - c.z};
        const double nn[3] = {tg[3 * n + k], tg[4 * n + k], tg[5 * n + k]};
        const double w = wv[k], v = wv[n + k];
        double pw[NT];
        pw[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= P; ++q) {
#pragma unroll
            for (int k1 = q; k1 >= 0; --k1) {
#pragma unroll
                for (int k2 = q - k1; k2 >= 0; --k2) {
                    const int k3 = q - k1 - k2;
                    const int t = mi(k1, k2, k3);
                    if (k1 > 0)
                        pw[t] = pw[mi(k1 - 1, k2, k3)] * h[0];
                    else if (k2 > 0)
                        pw[t] = pw[mi(k1, k2 - 1, k3)] * h[1];
                    else
                        pw[t] = pw[mi(k1, k2, k3 - 1)] * h[2];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc[t] += w * pw[t];
            acc[NT + t] += v * nn[0] * pw[t];
            acc[2 * NT + t] += v * nn[1] * pw[t];
            acc[3 * NT + t] += v * nn[2] * pw[t];
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 4 * NT; ++t) {
        double s = acc[t];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            s += __shfl_down(s, off, 64);
        if (lane == 0)
            red[wid][t] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 4 * NT; t += TPB)
        mom[(int64_t)blockIdx.x * 4 * NT + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// One pair of the direct sum (kernels K1'..K4' written out), target i with
// normal ni, source at separation d = x_i - x_j with normal nj and weights
// w = a psi, v = a phi.
__device__ __forceinline__ void pair_direct(const double d[3], const double ni[3],
                                            const double nj[3], double w, double v, double eps,
                                            double ieps, double kappa, double &s1, double &s2)
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double ir = rsqrt_pos(r2);
    const double rho = r2 * ir;
    const double e = exp_neg_pair(kappa * rho);
    const double tp2 = (1.0 + kappa * rho) * e;
    const double ir2 = ir * ir, ir3 = ir2 * ir;
    const double cx = ni[0] * d[0] + ni[1] * d[1] + ni[2] * d[2];
    const double cy = nj[0] * d[0] + nj[1] * d[1] + nj[2] * d[2];
    const double nn = ni[0] * nj[0] + ni[1] * nj[1] + ni[2] * nj[2];
    const double k1 = ir - e * ir;
    const double k2 = (eps * tp2 - 1.0) * cy * ir3;
    const double k3 = (tp2 * ieps - 1.0) * cx * ir3;
    const double h0 = (nn - 3.0 * cx * cy * ir2) * ir3;
    const double k4 = (tp2 - 1.0) * h0 - kappa * kappa * cx * cy * ir2 * e * ir;
    s1 += k1 * w + k2 * v;
    s2 += k3 * w + k4 * v;
}

// Far field of one cluster on one target: coefficients of both kernels to
// order P + 2 by the recurrences, each consumed as soon as it is formed.
// 1/eps (ieps) and 1/q enter as multiplications: an FP64 division is a
// sequence of about ten dependent instructions here, and the walk runs one
// wave per SIMD, with nothing else to hide their latency.
template <int P>
__device__ __forceinline__ void far_field(const double R[3], const double ni[3],
                                          const double *__restrict__ mo, double eps,
                                          double ieps, double kappa, double &s1, double &s2)
{
    constexpr int Q = P + 2;
    constexpr int NQ = nterms(Q);
    constexpr int NT = nterms(P);
    const double *M = mo, *D = mo + NT;   // D_d^k at D[d * NT + k]
    double A0[NQ], A[NQ], B[NQ];
    const double rho2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    const double irho2 = 1.0 / rho2;
    const double irho = sqrt(irho2);
    const double e = exp_neg_pair(kappa * rho2 * irho);
    A0[0] = irho;
    A[0] = e * irho;
    B[0] = e;
    s1 += (A0[0] - A[0]) * M[0];
#pragma unroll
    for (int q = 1; q <= Q; ++q) {
        const double rq = 1.0 / q;   // a constant once the loop is unrolled
        const double iq = irho2 * rq;
#pragma unroll
        for (int k1 = q; k1 >= 0; --k1) {
#pragma unroll
            for (int k2 = q - k1; k2 >= 0; --k2) {
                const int k3 = q - k1 - k2;
                const int m[3] = {k1, k2, k3};
                const int t = mi(k1, k2, k3);
                double l0 = 0.0, l = 0.0, lb = 0.0, g0 = 0.0, g = 0.0, gb = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    if (m[i] >= 1) {
                        const int u = mi(k1 - (i == 0), k2 - (i == 1), k3 - (i == 2));
                        l0 += R[i] * A0[u];
                        l += R[i] * A[u];
                        lb += R[i] * B[u];
                    }
                    if (m[i] >= 2) {
                        const int u = mi(k1 - 2 * (i == 0), k2 - 2 * (i == 1), k3 - 2 * (i == 2));
                        g0 += A0[u];
                        g += A[u];
                        gb += B[u];
                    }
                }
                A0[t] = ((2 * q - 1) * l0 - (q - 1) * g0) * iq;
                A[t] = ((2 * q - 1) * l - (q - 1) * g + kappa * (lb - gb)) * iq;
                B[t] = kappa * (l - g) * rq;
                // consume T^m (T0 = A0, Tk = A) at m = (k1, k2, k3)
                if (q <= P)   // K1 on the psi moments
                    s1 += (A0[t] - A[t]) * M[t];
                if (q <= P + 1) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (m[d] >= 1) {
                            const int u = mi(k1 - (d == 0), k2 - (d == 1), k3 - (d == 2));
                            // K2: source normal derivative on the phi moments
                            s1 += m[d] * (eps * A[t] - A0[t]) * D[d * NT + u];
                            // K3: target normal derivative on the psi moments
                            s2 -= m[d] * ni[d] * (A0[t] - A[t] * ieps) * M[u];
                        }
                    }
                }
#pragma unroll
                for (int ee = 0; ee < 3; ++ee) {
                    if (m[ee] < 1)
                        continue;
                    const int me[3] = {k1 - (ee == 0), k2 - (ee == 1), k3 - (ee == 2)};
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (me[d] < 1)
                            continue;
                        // K4: both derivatives on the phi moments
                        const int u = mi(me[0] - (d == 0), me[1] - (d == 1), me[2] - (d == 2));
                        s2 -= m[ee] * me[d] * ni[ee] * (A[t] - A0[t]) * D[d * NT + u];
                    }
                }
            }
        }
    }
}

// One thread per target (tree order): walk the tree once.
template <int P>
__global__ __launch_bounds__(TPB) void kt_eval(const TreeNode *__restrict__ nodes,
                                               const double4 *__restrict__ ctr, int n_nodes,
                                               const double *__restrict__ tg, int64_t n,
                                               const double *__restrict__ wv,
                                               const double *__restrict__ mom, double theta,
                                               double eps, double kappa,
                                               double *__restrict__ out,
                                               int64_t *__restrict__ counts)
{
    constexpr int NT = nterms(P);
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const double xi[3] = {tg[i], tg[n + i], tg[2 * n + i]};
    const double ni[3] = {tg[3 * n + i], tg[4 * n + i], tg[5 * n + i]};
    const double ieps = 1.0 / eps;
    double s1 = 0.0, s2 = 0.0;
    int64_t n_far = 0, n_pairs = 0;
    int node = 0;
    while (node < n_nodes) {
        const TreeNode nd = nodes[node];
        const double4 c = ctr[node];
        const double R[3] = {xi[0] - c.x, xi[1] - c.y, xi[2] - c.z};
        const double R2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        if (R2 > 0.0 && c.w <= theta * sqrt(R2)) {
            far_field<P>(R, ni, mom + (int64_t)node * 4 * NT, eps, ieps, kappa, s1, s2);
            ++n_far;
            node = nd.next;
        } else if (nd.leaf) {
            for (int j = nd.lo; j < nd.hi; ++j) {
                if (j == (int)i)
                    continue;
                const double d[3] = {xi[0] - tg[j], xi[1] - tg[n + j], xi[2] - tg[2 * n + j]};
                const double nj[3] = {tg[3 * n + j], tg[4 * n + j], tg[5 * n + j]};
                pair_direct(d, ni, nj, wv[j], wv[n + j], eps, ieps, kappa, s1, s2);
            }
            n_pairs += nd.hi - nd.lo - ((int)i >= nd.lo && (int)i < nd.hi);
            node = nd.next;
        } else {
            node = node + 1;   // first child
        }
    }
    out[i] = s1;
    out[n + i] = s2;
    if (counts) {
        counts[i] = n_far;
        counts[n + i] = n_pairs;
    }
}

// y = diag x - (1/4pi) s, back in the original order.
__global__ __launch_bounds__(TPB) void kt_finish(const int32_t *__restrict__ perm, int64_t n,
                                                 const double *__restrict__ out,
                                                 const double *__restrict__ x, double alpha,
                                                 double beta, double *__restrict__ y)
{
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k >= n)
        return;
    const int32_t i = perm[k];
    y[i] = alpha * x[i] - INV_4PI * out[k];
    y[n + i] = beta * x[n + i] - INV_4PI * out[n + k];
}

// Permuted target geometry: x, y, z, nx, ny, nz in tree order.
__global__ __launch_bounds__(TPB) void kt_permute(const int32_t *__restrict__ perm, int64_t n,
                                                  const double *__restrict__ g, int64_t npad,
                                                  double *__restrict__ tg)
{
    const int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (k >= n)
        return;
    const int32_t i = perm[k];
#pragma unroll
    for (int a = 0; a < 6; ++a)
        tg[a * n + k] = g[a * npad + i];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

// ---- host: tree --------------------------------------------------------------

// Depth-first octree with the subdivision rule described above.  Fills the
// point permutation and, per node, (lo, hi, next, leaf) and (centre, r_c).
void build_tree(const double *x, const double *y, const double *z, int64_t n, int n0,
                std::vector<int32_t> &perm, std::vector<int32_t> &node_i,
                std::vector<double> &node_d)
{
    double lo[3] = {x[0], y[0], z[0]}, hi[3] = {x[0], y[0], z[0]};
    for (int64_t i = 1; i < n; ++i) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    double c0[3], h0 = 0.0;
    for (int k = 0; k < 3; ++k) {
        c0[k] = 0.5 * (lo[k] + hi[k]);
        h0 = std::max(h0, 0.5 * (hi[k] - lo[k]));
    }
    perm.clear();
    node_i.clear();
    node_d.clear();
    struct Rec {
        static void go(const double *x, const double *y, const double *z, int n0,
                       std::vector<int32_t> &idx, const double c[3], double h, int depth,
                       std::vector<int32_t> &perm, std::vector<int32_t> &node_i,
                       std::vector<double> &node_d)
        {
            const int me = (int)(node_i.size() / 4);
            double blo[3] = {x[idx[0]], y[idx[0]], z[idx[0]]}, bhi[3] = {blo[0], blo[1], blo[2]};
            for (int32_t i : idx) {
                const double p[3] = {x[i], y[i], z[i]};
                for (int k = 0; k < 3; ++k) {
                    blo[k] = std::min(blo[k], p[k]);
                    bhi[k] = std::max(bhi[k], p[k]);
                }
            }
            const double dx = bhi[0] - blo[0], dy = bhi[1] - blo[1], dz = bhi[2] - blo[2];
            node_i.insert(node_i.end(), {(int32_t)perm.size(), 0, 0, 0});
            node_d.insert(node_d.end(), {0.5 * (blo[0] + bhi[0]), 0.5 * (blo[1] + bhi[1]),
                                         0.5 * (blo[2] + bhi[2]),
                                         0.5 * std::sqrt(dx * dx + dy * dy + dz * dz)});
            if ((int64_t)idx.size() <= n0 || depth >= 40) {
                perm.insert(perm.end(), idx.begin(), idx.end());
                node_i[4 * me + 3] = 1;
            } else {
                std::vector<int32_t> sub[8];
                for (int32_t i : idx) {
                    const int o = (x[i] >= c[0] ? 1 : 0) + (y[i] >= c[1] ? 2 : 0) +
                                  (z[i] >= c[2] ? 4 : 0);
                    sub[o].push_back(i);
                }
                idx.clear();
                idx.shrink_to_fit();
                for (int o = 0; o < 8; ++o) {
                    if (sub[o].empty())
                        continue;
                    const double hh = 0.5 * h;
                    const double cc[3] = {c[0] + ((o & 1) ? hh : -hh), c[1] + ((o & 2) ? hh : -hh),
                                          c[2] + ((o & 4) ? hh : -hh)};
                    go(x, y, z, n0, sub[o], cc, hh, depth + 1, perm, node_i, node_d);
                }
            }
            node_i[4 * me + 1] = (int32_t)perm.size();
            node_i[4 * me + 2] = (int32_t)(node_i.size() / 4);   // next: after the subtree
        }
    };
    std::vector<int32_t> all(n);
    for (int64_t i = 0; i < n; ++i)
        all[i] = (int32_t)i;
    Rec::go(x, y, z, n0, all, c0, h0, 0, perm, node_i, node_d);
}

// ---- host: the tree of the context's geometry, then treecode matvecs -------------

// Builds (or keeps) the tree of the current geometry with leaves of at most
// n0 points, and the permuted geometry.
int tree_prepare(pb_ctx *c, int n0)
{
    if (c->t_ready && c->t_n0 == n0)
        return PB_OK;
    const Geo &g = c->g;
    const int64_t n = g.n;
    std::vector<double> h(3 * g.npad);
    HIPCHK(hipMemcpyAsync(h.data(), g.g, sizeof(double) * 3 * g.npad, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<int32_t> perm, node_i;
    std::vector<double> node_d;
    build_tree(h.data(), h.data() + g.npad, h.data() + 2 * g.npad, n, n0, perm, node_i, node_d);
    const int n_nodes = (int)(node_i.size() / 4);
    TRY(ensure(c, c->t_nodes, sizeof(int32_t) * node_i.size()));
    TRY(ensure(c, c->t_ctr, sizeof(double) * node_d.size()));
    TRY(ensure(c, c->t_perm, sizeof(int32_t) * n));
    TRY(ensure(c, c->t_geo, sizeof(double) * 6 * n));
    TRY(ensure(c, c->t_wv, sizeof(double) * 2 * n));
    TRY(ensure(c, c->t_out, sizeof(double) * 2 * n));
    HIPCHK(hipMemcpyAsync(c->t_nodes.p, node_i.data(), sizeof(int32_t) * node_i.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->t_ctr.p, node_d.data(), sizeof(double) * node_d.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->t_perm.p, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice,
                          c->stream));
    hipLaunchKernelGGL(kt_permute, dim3(nblk(n)), dim3(TPB), 0, c->stream,
                       as<int32_t>(c->t_perm), n, g.g, g.npad, as<double>(c->t_geo));
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(c->stream));   // host vectors go out of scope
    c->t_n_nodes = n_nodes;
    c->t_n0 = n0;
    c->t_ready = true;
    return PB_OK;
}

// y = A x with the treecode (needs tree_prepare for the current geometry).
int tree_apply(pb_ctx *c, const pb_params *p, double theta, int order, const double *x,
               double *y, int64_t *counts)
{
    const Geo &g = c->g;
    const int64_t n = g.n;
    const int n_nodes = c->t_n_nodes;
    const int NT = nterms(order);
    TRY(ensure(c, c->t_mom, sizeof(double) * 4 * NT * (size_t)n_nodes));
    if (counts)
        TRY(ensure(c, c->t_cnt, sizeof(int64_t) * 2 * n));
    const auto *nodes = as<TreeNode>(c->t_nodes);
    const auto *ctr = as<double4>(c->t_ctr);
    const int32_t *dperm = as<int32_t>(c->t_perm);
    double *tg = as<double>(c->t_geo), *wv = as<double>(c->t_wv), *out = as<double>(c->t_out);
    double *mom = as<double>(c->t_mom);
    hipLaunchKernelGGL(kt_gather, dim3(nblk(n)), dim3(TPB), 0, c->stream, dperm, n,
                       g.g + 6 * g.npad, x, wv);
    LAUNCHCHK();
    const double eps = p->eps_out / p->eps_in, kap = p->kappa;
    int64_t *cnt = counts ? as<int64_t>(c->t_cnt) : nullptr;
    {
        ProfScope ps(c, PB_KERNEL_TREE, (double)n * (double)(n - 1));
#define PB_TREE_CASE(PP)                                                                        \
    case PP:                                                                                    \
        hipLaunchKernelGGL(kt_moments<PP>, dim3(n_nodes), dim3(TPB), 0, c->stream, nodes, ctr, \
                           tg, n, wv, mom);                                                     \
        hipLaunchKernelGGL(kt_eval<PP>, dim3(nblk(n)), dim3(TPB), 0, c->stream, nodes, ctr,    \
                           n_nodes, tg, n, wv, mom, theta, eps, kap, out, cnt);                 \
        break;
        switch (order) {
            PB_TREE_CASE(0)
            PB_TREE_CASE(1)
            PB_TREE_CASE(2)
            PB_TREE_CASE(3)
            PB_TREE_CASE(4)
            PB_TREE_CASE(5)
        default:
            return fail(c, PB_ERR_ARG, "treecode order must be 0..5");
        }
#undef PB_TREE_CASE
    }
    LAUNCHCHK();
    hipLaunchKernelGGL(kt_finish, dim3(nblk(n)), dim3(TPB), 0, c->stream, dperm, n, out, x,
                       0.5 * (1.0 + eps), 0.5 * (1.0 + 1.0 / eps), y);
    LAUNCHCHK();
    if (counts) {
        std::vector<int64_t> hc(2 * n);
        HIPCHK(hipMemcpyAsync(hc.data(), cnt, sizeof(int64_t) * 2 * n, hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        counts[0] = counts[1] = 0;
        for (int64_t k = 0; k < n; ++k) {
            counts[0] += hc[k];
            counts[1] += hc[n + k];
        }
        counts[2] = n_nodes;
    }
    return PB_OK;
}

int tree_matvec(pb_ctx *c, const pb_params *p, double theta, int order, int n0, const double *x,
                double *y, int64_t *counts)
{
    TRY(tree_prepare(c, n0));
    return tree_apply(c, p, theta, order, x, y, counts);
}

}  // namespace pbk
