/*
 * A plain C (C99) caller of the library through include/pbsolve.h alone: no
 * HIP, no Python.  Reads one system from a binary file, solves it in FP64 and
 * in refined FP32 with the leaf preconditioner, computes its charge
 * derivatives, checks an error path, and prints one "key value" pair per line.
 *
 * Input file (native byte order):
 *   int64 n_vert, n_tri, n_charges
 *   double eps_in, eps_out, kappa
 *   double vert[n_vert][3]; int32 tri[n_tri][3]; double pos[n_charges][3]; double q[n_charges]
 *
 * Exit status 0 when every call returned PB_OK, 1 on bad input, 2 on a
 * library error (its message is printed).
 */
#include "pbsolve.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int read_all(FILE *f, void *p, size_t size, size_t n)
{
    return n == 0 || fread(p, size, n, f) == n;
}

static int check(pb_ctx *ctx, int rc, const char *what)
{
    if (rc != PB_OK) {
        printf("error %s %d %s\n", what, rc, pb_last_error(ctx));
        return 0;
    }
    return 1;
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: %s input.bin\n", argv[0]);
        return 1;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) {
        perror(argv[1]);
        return 1;
    }
    int64_t dims[3];
    double phys[3];
    if (!read_all(f, dims, sizeof dims[0], 3) || !read_all(f, phys, sizeof phys[0], 3) ||
        dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) {
        fprintf(stderr, "bad header\n");
        fclose(f);
        return 1;
    }
    const int64_t nv = dims[0], nt = dims[1], nc = dims[2];
    double *vert = malloc(sizeof(double) * 3 * (size_t)nv);
    int32_t *tri = malloc(sizeof(int32_t) * 3 * (size_t)nt);
    double *pos = malloc(sizeof(double) * 3 * (size_t)nc);
    double *q = malloc(sizeof(double) * (size_t)nc);
    double *phi = malloc(sizeof(double) * (size_t)nt);
    double *dphi = malloc(sizeof(double) * (size_t)nt);
    double *de_dpos = malloc(sizeof(double) * 3 * (size_t)nc);
    double *de_dq = malloc(sizeof(double) * (size_t)nc);
    int ok = vert && tri && pos && q && phi && dphi && de_dpos && de_dq &&
             read_all(f, vert, sizeof(double), 3 * (size_t)nv) &&
             read_all(f, tri, sizeof(int32_t), 3 * (size_t)nt) &&
             read_all(f, pos, sizeof(double), 3 * (size_t)nc) &&
             read_all(f, q, sizeof(double), (size_t)nc);
    fclose(f);
    if (!ok) {
        fprintf(stderr, "short input\n");
        return 1;
    }

    pb_ctx *ctx = NULL;
    int status = 0;
    const int rc_create = pb_create(0, NULL, &ctx);
    if (rc_create != PB_OK) {
        printf("error create %d %s\n", rc_create, ctx ? pb_last_error(ctx) : "");
        return 2;
    }
    printf("abi %d\n", pb_abi_version());

    const pb_surface s = {nv, nt, vert, tri};
    const pb_charges c = {nc, pos, q};
    pb_params p;
    memset(&p, 0, sizeof p);
    p.eps_in = phys[0];
    p.eps_out = phys[1];
    p.kappa = phys[2];
    p.restart = 10;
    p.max_iter = 1000;
    p.max_refine = 20;

    pb_info info;
    p.tol = 1e-10;
    p.precision = PB_FP64;
    if (check(ctx, pb_solve(ctx, &s, &c, &p, phi, dphi, &info), "solve_fp64"))
        printf("e_fp64 %.17g\niters_fp64 %d\n", info.e_solv, info.iters);
    else
        status = 2;

    double e_energy = 0.0;
    if (check(ctx, pb_energy(ctx, &s, &c, &p, phi, dphi, &e_energy), "energy"))
        printf("e_energy %.17g\n", e_energy);
    else
        status = 2;

    p.tol = 1e-8;
    p.precision = PB_FP32_IR;
    p.inner_tol = 1e-4;
    p.precond_leaf = 16;
    if (check(ctx, pb_solve(ctx, &s, &c, &p, NULL, NULL, &info), "solve_fp32ir"))
        printf("e_fp32ir %.17g\nmatvecs_fp32 %d\nmatvecs_fp64 %d\n", info.e_solv,
               info.matvecs_fp32, info.matvecs_fp64);
    else
        status = 2;

    p.tol = 1e-10;
    p.precision = PB_FP64;
    p.precond_leaf = 0;
    if (check(ctx, pb_forces(ctx, &s, &c, &p, de_dpos, de_dq, &info), "forces")) {
        printf("e_forces %.17g\n", info.e_solv);
        for (int64_t k = 0; k < nc; ++k)
            printf("de_dq %lld %.17g\nde_dpos %lld %.17g %.17g %.17g\n", (long long)k, de_dq[k],
                   (long long)k, de_dpos[3 * k], de_dpos[3 * k + 1], de_dpos[3 * k + 2]);
    } else {
        status = 2;
    }

    /* an error path: a negative tolerance is an argument error with a message */
    p.tol = -1.0;
    const int rc_bad = pb_solve(ctx, &s, &c, &p, NULL, NULL, &info);
    printf("bad_tol_status %d\nbad_tol_message %s\n", rc_bad, pb_last_error(ctx));

    pb_destroy(ctx);
    free(vert);
    free(tri);
    free(pos);
    free(q);
    free(phi);
    free(dphi);
    free(de_dpos);
    free(de_dq);
    return status;
}
