/*
 * FP64 CPU oracle for the direct-sum boundary-integral (DSBI) Poisson-
 * Boltzmann path.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
 * CPU-baseline leg of the benchmark may call this file; the product path
 * never does.  It shares no code with the HIP library.
 *
 * Everything is written as the plain definition: the Green's functions of
 * Sec. 2.2.1 (eq. eq_potential) and their normal derivatives obtained from
 * the chain rule on the radial profile G(rho), the kernels K1..K4 as the
 * combinations of eqs. Eq_K1/Eq_K2, the centroid-collocation sums of eqs.
 * eqbim_5/eqbim_6 with the j = i term skipped by index, the source terms of
 * eq. source_terms and the solvation-energy quadrature of eq.
 * solvation_energy.  No blocking, no fusion, no algebraic simplification.
 *
 * Sign convention (the paper's printed signs for the x-derivatives are
 * inconsistent): d/dnu_x = +nu(x).grad_x and the mixed derivative is
 * +sum_mn nu_m(x) nu_n(y) d_{x_m} d_{y_n} G.  This is the reading that makes
 * eqs. eqbim_3/eqbim_4 hold for the exact sphere solution.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static const double FOUR_PI = 12.566370614359172953850573533118; /* 4*pi */

/* Radial profile G(r) = exp(-kappa r)/(4 pi r) and its first two
 * derivatives with respect to r.  kappa = 0 gives the Coulomb G0. */
static void radial(double r, double kappa, double *g, double *g1, double *g2)
{
    double e = exp(-kappa * r);
    *g = e / (FOUR_PI * r);
    *g1 = -(1.0 + kappa * r) * e / (FOUR_PI * r * r);
    *g2 = (kappa * kappa * r * r + 2.0 * (1.0 + kappa * r)) * e / (FOUR_PI * r * r * r);
}

/* Value, gradients and mixed Hessian of G(x, y) = G(|x - y|).
 *   grad_x G = G'(r) d / r                      (d = x - y)
 *   grad_y G = -grad_x G
 *   H[m][n] = d_{x_m} d_{y_n} G = -[G'' d_m d_n / r^2 + G' (delta_mn / r - d_m d_n / r^3)]
 */
static void green_all(const double *x, const double *y, double kappa,
                      double *g, double gx[3], double H[3][3])
{
    double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double g0, g1, g2;
    radial(r, kappa, &g0, &g1, &g2);
    *g = g0;
    for (int m = 0; m < 3; ++m)
        gx[m] = g1 * d[m] / r;
    if (H) {
        for (int m = 0; m < 3; ++m)
            for (int n = 0; n < 3; ++n) {
                double delta = (m == n) ? 1.0 : 0.0;
                H[m][n] = -(g2 * d[m] * d[n] / (r * r)
                            + g1 * (delta / r - d[m] * d[n] / (r * r * r)));
            }
    }
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* G, dG/dnu_y, dG/dnu_x, d2G/dnu_x dnu_y for one pair. */
static void green_normal(const double *x, const double *nx, const double *y,
                         const double *ny, double kappa, double out[4])
{
    double g, gx[3], H[3][3];
    green_all(x, y, kappa, &g, gx, H);
    double gy[3] = {-gx[0], -gx[1], -gx[2]};
    double Hny[3];
    for (int m = 0; m < 3; ++m)
        Hny[m] = H[m][0] * ny[0] + H[m][1] * ny[1] + H[m][2] * ny[2];
    out[0] = g;
    out[1] = dot3(ny, gy);
    out[2] = dot3(nx, gx);
    out[3] = dot3(nx, Hny);
}

/* K1..K4 of eqs. Eq_K1/Eq_K2 (with the 1/(4 pi) of the Green's functions). */
static void kernels(const double *x, const double *nx, const double *y,
                    const double *ny, double eps, double kappa, double K[4])
{
    double a0[4], ak[4];
    green_normal(x, nx, y, ny, 0.0, a0);
    green_normal(x, nx, y, ny, kappa, ak);
    K[0] = a0[0] - ak[0];
    K[1] = eps * ak[1] - a0[1];
    K[2] = a0[2] - ak[2] / eps;
    K[3] = ak[3] - a0[3];
}

/* ---- exported entry points ------------------------------------------- */

void orc_green(const double *x, const double *nx, const double *y,
               const double *ny, double kappa, double *out4)
{
    green_normal(x, nx, y, ny, kappa, out4);
}

void orc_kernels(const double *x, const double *nx, const double *y,
                 const double *ny, double eps, double kappa, double *out4)
{
    kernels(x, nx, y, ny, eps, kappa, out4);
}

/* Centroid-collocation matvec, eqs. eqbim_5/eqbim_6 with unknowns
 * [phi; psi] (psi = dphi/dnu), area weights on the source side:
 *   y1_i = (1+eps)/2 phi_i - sum_{j != i} [K1_ij psi_j + K2_ij phi_j] a_j
 *   y2_i = (1+1/eps)/2 psi_i - sum_{j != i} [K3_ij psi_j + K4_ij phi_j] a_j
 * Rows listed in rows[0..nrows) (all rows when rows == NULL).  abs1/abs2
 * (may be NULL) receive the sum of absolute values of every term. */
void orc_matvec(int64_t n, const double *cen, const double *nrm, const double *area,
                double eps, double kappa, const double *phi, const double *psi,
                int64_t nrows, const int64_t *rows, double *y1, double *y2,
                double *abs1, double *abs2)
{
    int64_t m = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        double s1 = 0.0, s2 = 0.0, b1 = 0.0, b2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double K[4];
            kernels(cen + 3 * i, nrm + 3 * i, cen + 3 * j, nrm + 3 * j, eps, kappa, K);
            double t1 = K[0] * psi[j] * area[j], t2 = K[1] * phi[j] * area[j];
            double t3 = K[2] * psi[j] * area[j], t4 = K[3] * phi[j] * area[j];
            s1 += t1 + t2;
            s2 += t3 + t4;
            b1 += fabs(t1) + fabs(t2);
            b2 += fabs(t3) + fabs(t4);
        }
        double d1 = 0.5 * (1.0 + eps) * phi[i];
        double d2 = 0.5 * (1.0 + 1.0 / eps) * psi[i];
        y1[r] = d1 - s1;
        y2[r] = d2 - s2;
        if (abs1) abs1[r] = fabs(d1) + b1;
        if (abs2) abs2[r] = fabs(d2) + b2;
    }
}

/* Transpose of the matvec above.  With (M_k)_ij = K_k(x_i, x_j) a_j and
 * A = [[aI - M2, -M1], [-M4, bI - M3]]:
 *   (A^T l)1_i = a l1_i - sum_{j != i} [K2(x_j,x_i) l1_j + K4(x_j,x_i) l2_j] a_i
 *   (A^T l)2_i = b l2_i - sum_{j != i} [K1(x_j,x_i) l1_j + K3(x_j,x_i) l2_j] a_i */
void orc_matvec_t(int64_t n, const double *cen, const double *nrm, const double *area,
                  double eps, double kappa, const double *l1, const double *l2,
                  int64_t nrows, const int64_t *rows, double *y1, double *y2,
                  double *abs1, double *abs2)
{
    int64_t m = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        double s1 = 0.0, s2 = 0.0, b1 = 0.0, b2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double K[4];
            kernels(cen + 3 * j, nrm + 3 * j, cen + 3 * i, nrm + 3 * i, eps, kappa, K);
            double t1 = K[1] * l1[j] * area[i], t2 = K[3] * l2[j] * area[i];
            double t3 = K[0] * l1[j] * area[i], t4 = K[2] * l2[j] * area[i];
            s1 += t1 + t2;
            s2 += t3 + t4;
            b1 += fabs(t1) + fabs(t2);
            b2 += fabs(t3) + fabs(t4);
        }
        double d1 = 0.5 * (1.0 + eps) * l1[i];
        double d2 = 0.5 * (1.0 + 1.0 / eps) * l2[i];
        y1[r] = d1 - s1;
        y2[r] = d2 - s2;
        if (abs1) abs1[r] = fabs(d1) + b1;
        if (abs2) abs2[r] = fabs(d2) + b2;
    }
}

/* Dense 2n x 2n matrix of the matvec, row-major, block layout [phi; psi]. */
void orc_assemble(int64_t n, const double *cen, const double *nrm, const double *area,
                  double eps, double kappa, double *A)
{
    int64_t n2 = 2 * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double K[4] = {0.0, 0.0, 0.0, 0.0};
            if (j != i)
                kernels(cen + 3 * i, nrm + 3 * i, cen + 3 * j, nrm + 3 * j, eps, kappa, K);
            A[i * n2 + j] = -K[1] * area[j];
            A[i * n2 + n + j] = -K[0] * area[j];
            A[(n + i) * n2 + j] = -K[3] * area[j];
            A[(n + i) * n2 + n + j] = -K[2] * area[j];
        }
        A[i * n2 + i] += 0.5 * (1.0 + eps);
        A[(n + i) * n2 + n + i] += 0.5 * (1.0 + 1.0 / eps);
    }
}

/* Rows and columns idx[0..m) of the dense matrix, as a 2m x 2m block in
 * the same [phi; psi] block layout (the leaf blocks of the preconditioner of
 * Sec. 2.2.4). */
void orc_assemble_subset(int64_t n, const double *cen, const double *nrm, const double *area,
                         double eps, double kappa, int64_t m, const int64_t *idx, double *B)
{
    (void)n;
    int64_t m2 = 2 * m;
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = idx[r];
        for (int64_t q = 0; q < m; ++q) {
            int64_t j = idx[q];
            double K[4] = {0.0, 0.0, 0.0, 0.0};
            if (j != i)
                kernels(cen + 3 * i, nrm + 3 * i, cen + 3 * j, nrm + 3 * j, eps, kappa, K);
            B[r * m2 + q] = -K[1] * area[j];
            B[r * m2 + m + q] = -K[0] * area[j];
            B[(m + r) * m2 + q] = -K[3] * area[j];
            B[(m + r) * m2 + m + q] = -K[2] * area[j];
        }
        B[r * m2 + r] += 0.5 * (1.0 + eps);
        B[(m + r) * m2 + m + r] += 0.5 * (1.0 + 1.0 / eps);
    }
}

/* Source terms, eq. source_terms:
 *   S1_i = (1/eps_in) sum_k q_k G0(x_i, y_k)
 *   S2_i = (1/eps_in) sum_k q_k dG0(x_i, y_k)/dnu_x */
void orc_source(int64_t n, const double *cen, const double *nrm, int64_t nc,
                const double *pos, const double *q, double eps_in,
                int64_t nrows, const int64_t *rows, double *s1, double *s2)
{
    int64_t m = rows ? nrows : n;
    double zero[3] = {0.0, 0.0, 0.0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        double a = 0.0, b = 0.0;
        for (int64_t k = 0; k < nc; ++k) {
            double o[4];
            green_normal(cen + 3 * i, nrm + 3 * i, pos + 3 * k, zero, 0.0, o);
            a += q[k] * o[0];
            b += q[k] * o[2];
        }
        s1[r] = a / eps_in;
        s2[r] = b / eps_in;
    }
}

/* Reaction potential at each charge, the integral of eq. solvation_energy:
 *   P_k = sum_j [K1(y_k, x_j) psi_j + K2(y_k, x_j) phi_j] a_j
 * and (when grad != NULL) its gradient with respect to y_k. */
void orc_reaction(int64_t n, const double *cen, const double *nrm, const double *area,
                  double eps, double kappa, const double *phi, const double *psi,
                  int64_t nc, const double *pos, double *P, double *grad)
{
    double zero[3] = {0.0, 0.0, 0.0};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nc; ++k) {
        const double *y = pos + 3 * k;
        double s = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            double K[4];
            kernels(y, zero, cen + 3 * j, nrm + 3 * j, eps, kappa, K);
            s += (K[0] * psi[j] + K[1] * phi[j]) * area[j];
            if (grad) {
                /* gradient with respect to the first argument of
                 * K1 = G0 - Gk and K2 = eps dGk/dnu_y - dG0/dnu_y */
                double g0, gx0[3], H0[3][3], gk, gxk[3], Hk[3][3];
                green_all(y, cen + 3 * j, 0.0, &g0, gx0, H0);
                green_all(y, cen + 3 * j, kappa, &gk, gxk, Hk);
                const double *nj = nrm + 3 * j;
                for (int m = 0; m < 3; ++m) {
                    double dK1 = gx0[m] - gxk[m];
                    double Hk_n = Hk[m][0] * nj[0] + Hk[m][1] * nj[1] + Hk[m][2] * nj[2];
                    double H0_n = H0[m][0] * nj[0] + H0[m][1] * nj[1] + H0[m][2] * nj[2];
                    double dK2 = eps * Hk_n - H0_n;
                    g[m] += (dK1 * psi[j] + dK2 * phi[j]) * area[j];
                }
            }
        }
        P[k] = s;
        if (grad) {
            grad[3 * k + 0] = g[0];
            grad[3 * k + 1] = g[1];
            grad[3 * k + 2] = g[2];
        }
    }
}

/* Adjoint right-hand side w = B^T q of E = 2 pi c_u q^T B xi:
 *   w1_j = sum_k q_k K2(y_k, x_j) a_j   (phi block)
 *   w2_j = sum_k q_k K1(y_k, x_j) a_j   (psi block) */
void orc_adjoint_rhs(int64_t n, const double *cen, const double *nrm, const double *area,
                     double eps, double kappa, int64_t nc, const double *pos,
                     const double *q, double *w1, double *w2)
{
    double zero[3] = {0.0, 0.0, 0.0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        double a = 0.0, b = 0.0;
        for (int64_t k = 0; k < nc; ++k) {
            double K[4];
            kernels(pos + 3 * k, zero, cen + 3 * j, nrm + 3 * j, eps, kappa, K);
            a += q[k] * K[1];
            b += q[k] * K[0];
        }
        w1[j] = a * area[j];
        w2[j] = b * area[j];
    }
}

/* Source-side adjoint terms for charge k:
 *   c_k = sum_i [l1_i S1col_ik + l2_i S2col_ik]
 *   g_k = sum_i [l1_i grad_{y_k} S1col_ik + l2_i grad_{y_k} S2col_ik]
 * with S1col_ik = G0(x_i, y_k)/eps_in and S2col_ik = dG0(x_i, y_k)/dnu_x / eps_in. */
void orc_source_adjoint(int64_t n, const double *cen, const double *nrm, double eps_in,
                        const double *l1, const double *l2, int64_t nc,
                        const double *pos, double *c, double *grad)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nc; ++k) {
        double s = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int64_t i = 0; i < n; ++i) {
            double g0, gx[3], H[3][3];
            const double *ni = nrm + 3 * i;
            green_all(cen + 3 * i, pos + 3 * k, 0.0, &g0, gx, H);
            s += l1[i] * g0 + l2[i] * dot3(ni, gx);
            for (int m = 0; m < 3; ++m) {
                /* grad_y G0 = -grad_x G0; grad_y (nu_x . grad_x G0) = H^T nu_x */
                double Htn = H[0][m] * ni[0] + H[1][m] * ni[1] + H[2][m] * ni[2];
                g[m] += l1[i] * (-gx[m]) + l2[i] * Htn;
            }
        }
        c[k] = s / eps_in;
        grad[3 * k + 0] = g[0] / eps_in;
        grad[3 * k + 1] = g[1] / eps_in;
        grad[3 * k + 2] = g[2] / eps_in;
    }
}

/* Coulomb potential of the charges, S1 of eq. source_terms at arbitrary
 * points: out_k = (1/eps_in) sum_l q_l G0(x_k, y_l), skipping l == k when
 * skip_self (x = the charge positions themselves). */
void orc_coulomb(int64_t npts, const double *pts, int64_t nc, const double *pos,
                 const double *q, double eps_in, int skip_self, double *out)
{
    double zero[3] = {0.0, 0.0, 0.0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npts; ++k) {
        double s = 0.0;
        for (int64_t l = 0; l < nc; ++l) {
            if (skip_self && l == k)
                continue;
            double o[4];
            green_normal(pts + 3 * k, zero, pos + 3 * l, zero, 0.0, o);
            s += q[l] * o[0];
        }
        out[k] = s / eps_in;
    }
}

