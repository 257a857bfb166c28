/* Every entry point of the oracle's C loops (oracle/dsbi_oracle.c) on a small
 * surface, built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_host_sanitizers.py (any report aborts the run).  The input file
 * holds n, nc, then cen [n][3], nrm [n][3], area [n], pos [nc][3], q [nc]
 * (little-endian int64 and double).  Besides running every loop, the program
 * prints the largest difference between the matvec loops and the dense
 * matrix of the same operator, which the test bounds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_matvec(int64_t n, const double *cen, const double *nrm, const double *area,
                double eps, double kappa, const double *phi, const double *psi,
                int64_t nrows, const int64_t *rows, double *y1, double *y2, double *abs1,
                double *abs2);
void orc_matvec_t(int64_t n, const double *cen, const double *nrm, const double *area,
                  double eps, double kappa, const double *l1, const double *l2, int64_t nrows,
                  const int64_t *rows, double *y1, double *y2, double *abs1, double *abs2);
void orc_assemble(int64_t n, const double *cen, const double *nrm, const double *area,
                  double eps, double kappa, double *A);
void orc_assemble_subset(int64_t n, const double *cen, const double *nrm, const double *area,
                         double eps, double kappa, int64_t m, const int64_t *idx, double *B);
void orc_source(int64_t n, const double *cen, const double *nrm, int64_t nc, const double *pos,
                const double *q, double eps_in, int64_t nrows, const int64_t *rows, double *s1,
                double *s2);
void orc_reaction(int64_t n, const double *cen, const double *nrm, const double *area,
                  double eps, double kappa, const double *phi, const double *psi, int64_t nc,
                  const double *pos, double *P, double *grad);
void orc_adjoint_rhs(int64_t n, const double *cen, const double *nrm, const double *area,
                     double eps, double kappa, int64_t nc, const double *pos, const double *q,
                     double *w1, double *w2);
void orc_source_adjoint(int64_t n, const double *cen, const double *nrm, double eps_in,
                        const double *l1, const double *l2, int64_t nc, const double *pos,
                        double *c, double *grad);
void orc_coulomb(int64_t npts, const double *pts, int64_t nc, const double *pos,
                 const double *q, double eps_in, int skip_self, double *out);

static double *take(FILE *f, size_t count)
{
    double *p = malloc(sizeof(double) * count);
    if (!p || fread(p, sizeof(double), count, f) != count) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2)
        return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f)
        return 2;
    int64_t hdr[2];
    if (fread(hdr, sizeof(int64_t), 2, f) != 2)
        return 2;
    const int64_t n = hdr[0], nc = hdr[1], n2 = 2 * hdr[0];
    double *cen = take(f, 3 * n), *nrm = take(f, 3 * n), *area = take(f, n);
    double *pos = take(f, 3 * nc), *q = take(f, nc);
    fclose(f);
    const double eps = 80.0, kappa = 0.1257;
    double *x = malloc(sizeof(double) * n2), *y = malloc(sizeof(double) * n2);
    double *ab = malloc(sizeof(double) * n2), *A = malloc(sizeof(double) * n2 * n2);
    for (int64_t i = 0; i < n2; ++i)
        x[i] = sin(0.37 * (double)i + 0.1);
    orc_assemble(n, cen, nrm, area, eps, kappa, A);
    double dmax = 0.0, amax = 0.0;
    for (int t = 0; t < 2; ++t) {
        if (t == 0)
            orc_matvec(n, cen, nrm, area, eps, kappa, x, x + n, n, NULL, y, y + n, ab, ab + n);
        else
            orc_matvec_t(n, cen, nrm, area, eps, kappa, x, x + n, n, NULL, y, y + n, ab, ab + n);
        for (int64_t r = 0; r < n2; ++r) {
            double s = 0.0;
            for (int64_t c = 0; c < n2; ++c)
                s += (t == 0 ? A[r * n2 + c] : A[c * n2 + r]) * x[c];
            dmax = fmax(dmax, fabs(s - y[r]));
            amax = fmax(amax, fabs(y[r]));
        }
    }
    printf("matvec_vs_dense %.6e\n", dmax / amax);
    /* a row subset gives the same rows */
    int64_t rows[3] = {0, n / 2, n - 1};
    double r1[3], r2[3];
    orc_matvec(n, cen, nrm, area, eps, kappa, x, x + n, 3, rows, r1, r2, NULL, NULL);
    orc_matvec(n, cen, nrm, area, eps, kappa, x, x + n, n, NULL, y, y + n, NULL, NULL);
    double dsub = 0.0;
    for (int k = 0; k < 3; ++k)
        dsub = fmax(dsub, fmax(fabs(r1[k] - y[rows[k]]), fabs(r2[k] - y[n + rows[k]])));
    printf("rows_subset %.6e\n", dsub);
    /* a leaf block is the dense matrix restricted to its indices */
    int64_t idx[4] = {1, 3, n / 3, n - 2};
    double B[64];
    orc_assemble_subset(n, cen, nrm, area, eps, kappa, 4, idx, B);
    double dblk = 0.0;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            const int64_t ra = a < 4 ? idx[a] : n + idx[a - 4];
            const int64_t cb = b < 4 ? idx[b] : n + idx[b - 4];
            dblk = fmax(dblk, fabs(B[a * 8 + b] - A[ra * n2 + cb]));
        }
    printf("subset_block %.6e\n", dblk);
    double *s1 = malloc(sizeof(double) * n), *s2 = malloc(sizeof(double) * n);
    orc_source(n, cen, nrm, nc, pos, q, 2.0, 0, NULL, s1, s2);
    double *P = malloc(sizeof(double) * nc), *G = malloc(sizeof(double) * 3 * nc);
    orc_reaction(n, cen, nrm, area, eps, kappa, x, x + n, nc, pos, P, G);
    orc_adjoint_rhs(n, cen, nrm, area, eps, kappa, nc, pos, q, s1, s2);
    orc_source_adjoint(n, cen, nrm, 2.0, x, x + n, nc, pos, P, G);
    orc_coulomb(nc, pos, nc, pos, q, 2.0, 1, P);
    double chk = 0.0;
    for (int64_t k = 0; k < nc; ++k)
        chk += P[k] + G[3 * k] + G[3 * k + 1] + G[3 * k + 2];
    for (int64_t i = 0; i < n; ++i)
        chk += s1[i] + s2[i];
    printf("finite %d\n", isfinite(chk) ? 1 : 0);
    free(cen), free(nrm), free(area), free(pos), free(q), free(x), free(y), free(ab), free(A);
    free(s1), free(s2), free(P), free(G);
    return 0;
}
