/*
 * pbsolve.h -- C ABI of the MI355X direct-sum boundary-integral (DSBI)
 * Poisson-Boltzmann library (libpbdsbi.so, HIP for gfx950).
 *
 * The library solves the well-conditioned boundary integral form of the
 * linearized Poisson-Boltzmann equation (Sec. 2.2.1, eqs. eqbim_3/eqbim_4)
 * discretized by centroid collocation on flat triangles (Sec. 2.2.2, eqs.
 * eqbim_5/eqbim_6, the singular j = i term omitted) with restarted GMRES,
 * and evaluates the electrostatic solvation energy (eq. solvation_energy).
 *
 * Conventions shared by every entry point
 *   - Sizes are int64_t, reals are double, arrays are row-major and
 *     C-contiguous.  Vectors of unknowns use block layout [phi; dphi]
 *     (length 2 n_tri): phi = surface potential, dphi = its normal
 *     derivative from inside.
 *   - Units: Angstrom, elementary charges, kcal/mol.  phi/dphi are the
 *     solution of eqs. eqbim_5/eqbim_6, i.e. the physical potential in e_c/A
 *     divided by 4 pi; multiply by 4 pi * 332.0716 for kcal/mol/e_c.
 *   - Triangles are listed counter-clockwise seen from the solvent side, so
 *     (v1-v0)x(v2-v0) is the outward normal.
 *   - Ownership: the caller owns every buffer it passes; the library never
 *     frees or keeps caller memory.  Device scratch belongs to the context
 *     and is reused across calls.
 *   - Host-pointer entry points copy inputs to the device and results back;
 *     *_dev entry points take device pointers, enqueue on the context's
 *     stream and return after that stream has drained.
 *   - Errors: every entry point returns a status (below); no exception
 *     crosses the ABI.  On a negative status outputs are unspecified and
 *     pb_last_error(ctx) describes the failure.
 *   - A context is used by one host thread at a time.
 */
#ifndef PBSOLVE_H
#define PBSOLVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PB_ABI_VERSION 1

/* status codes */
#define PB_OK 0
#define PB_NOT_CONVERGED 1      /* outputs hold the last iterate; info->rel_residual set */
#define PB_ERR_ARG (-1)         /* NULL pointer, n <= 0, eps <= 0, kappa outside [0, 100],
                                   tol <= 0, restart < 1 ... */
#define PB_ERR_GEOMETRY (-2)    /* non-finite vertex, index out of range, zero-area triangle,
                                   centroid coordinate beyond 1e5 A, two triangles with the
                                   same centroid (the singular j = i term is skipped by
                                   index, eqs. eqbim_5/eqbim_6), non-positive enclosed
                                   volume (wrong orientation); the message names the
                                   offending triangle where there is one */
#define PB_ERR_CHARGE (-3)      /* a charge outside the surface (discrete solid angle < 2 pi) */
#define PB_ERR_HIP (-4)         /* HIP runtime error */
#define PB_ERR_OOM (-5)         /* device allocation failed */

/* precision of the matvec inside GMRES */
#define PB_FP64 0               /* FP64 everywhere */
#define PB_FP32_IR 1            /* FP32 matvec in an inner GMRES, FP64 iterative refinement */

typedef struct pb_ctx pb_ctx;

/* Closed triangulated surface. vert: [n_vert][3]; tri: [n_tri][3] indices into vert. */
typedef struct {
    int64_t n_vert, n_tri;
    const double *vert;
    const int32_t *tri;
} pb_surface;

/* Point charges strictly inside the surface. pos: [n][3] (A); q: [n] (e_c). */
typedef struct {
    int64_t n;
    const double *pos;
    const double *q;
} pb_charges;

typedef struct {
    double eps_in, eps_out;     /* dielectric constants inside / outside (> 0) */
    double kappa;               /* inverse Debye length outside, 1/A (0 <= kappa <= 100) */
    double tol;                 /* relative residual |b - A x|_2 / |b|_2 at which to stop */
    int32_t restart;            /* GMRES restart length m (>= 1; the paper's runs use 10) */
    int32_t max_iter;           /* cap on Arnoldi steps (FP64) / outer refinements x inner cap (IR) */
    int32_t precision;          /* PB_FP64 or PB_FP32_IR */
    int32_t max_refine;         /* IR: cap on refinement steps */
    double inner_tol;           /* IR: relative tolerance of the first inner FP32 GMRES
                                   solve, in (0, 1) (PB_ERR_ARG otherwise; unused by
                                   PB_FP64).  A later correction solve, with outer residual
                                   r, stops at max(inner_tol, 0.3 tol |b| / |r|) (at most
                                   0.5): just enough to bring the outer residual under
                                   tol.  Values below 1e-7 (beyond what FP32 pair
                                   arithmetic resolves) are raised to 1e-7, and an inner
                                   solve also ends when a restart cycle gains less
                                   than 10 % */
    int32_t precond_leaf;       /* 0: no preconditioner.  1..100: block-diagonal leaf
                                   preconditioner of Sec. 2.2.4 with at most this many
                                   elements per octree leaf (N0; the paper's runs use
                                   100); GMRES then runs on the left-
                                   preconditioned system M^-1 A x = M^-1 b and tol applies
                                   to its residual |M^-1 (b - A x)| / |M^-1 b| (FP64 path,
                                   IR inner solves and IR outer test alike; the outer
                                   residual b - A x itself is formed in FP64). */
    int32_t reserved;           /* set to 0 */
} pb_params;

typedef struct {
    double e_solv;              /* solvation energy, kcal/mol */
    double rel_residual;        /* final relative residual (FP64); left-preconditioned
                                   when precond_leaf > 0 */
    double seconds;             /* wall time inside the call */
    int32_t iters;              /* Arnoldi steps (one matvec each), all precisions */
    int32_t matvecs_fp64;       /* FP64 matvecs, including residual checks */
    int32_t matvecs_fp32;       /* FP32 matvecs */
    int32_t refinements;        /* IR outer steps (0 for PB_FP64) */
    int32_t status;             /* same as the return value */
    int32_t adjoint_iters;      /* Arnoldi steps of the adjoint solve (pb_forces*) */
} pb_info;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on, or NULL for a stream the context creates (default priority). */
int pb_create(int device, void *hip_stream, pb_ctx **out);
void pb_destroy(pb_ctx *ctx);
/* Message for the last non-zero status returned on ctx (never NULL). */
const char *pb_last_error(const pb_ctx *ctx);
int pb_abi_version(void);

/* ---- host-pointer entry points ---------------------------------------- */

/* Step 1, collocation geometry (Sec. 2.2.2): centroid x_i = (v0+v1+v2)/3,
 * unit normal (v1-v0)x(v2-v0)/|.|, area |(v1-v0)x(v2-v0)|/2.
 * cen, nrm: [n_tri][3]; area: [n_tri].  Validates the surface (PB_ERR_GEOMETRY). */
int pb_geometry(pb_ctx *ctx, const pb_surface *s, double *cen, double *nrm, double *area);

/* Step 2, source terms (eq. source_terms): b = [S1; S2] at the centroids,
 * S1 = (1/eps_in) sum_k q_k G0(x_i, y_k), S2 = (1/eps_in) sum_k q_k dG0/dnu_x.
 * b: [2 n_tri]. */
int pb_source(pb_ctx *ctx, const pb_surface *s, const pb_charges *c, const pb_params *p,
              double *b);

/* Step 3 (and its transpose, step 6): y = A x for the system of eqs.
 * eqbim_5/eqbim_6, or y = A^T x when transpose != 0.  precision: PB_FP64 or
 * PB_FP32_IR (FP32 pair arithmetic, FP64 result).  x, y: [2 n_tri]. */
int pb_matvec(pb_ctx *ctx, const pb_surface *s, const pb_params *p, const double *x,
              double *y, int transpose, int precision);

/* Step 5, solvation energy (eq. solvation_energy) of a given surface
 * solution: E = (1/2) sum_k q_k phi_reac(y_k), in kcal/mol.
 * phi, dphi: [n_tri]. */
int pb_energy(pb_ctx *ctx, const pb_surface *s, const pb_charges *c, const pb_params *p,
              const double *phi, const double *dphi, double *e_solv);

/* Whole path: geometry, sources, restarted GMRES (FP64, or FP32 inner solves
 * with FP64 iterative refinement), energy.  phi/dphi ([n_tri] each) may be
 * NULL.  Returns PB_OK, PB_NOT_CONVERGED or a negative error. */
int pb_solve(pb_ctx *ctx, const pb_surface *s, const pb_charges *c, const pb_params *p,
             double *phi, double *dphi, pb_info *info);

/* Step 6 and the adjoint method: forward solve (as pb_solve), adjoint solve
 * A^T lam = B^T q with the transpose matvec (same precision and tolerance),
 * then the derivatives of E_sol for a fixed surface:
 *   dE_dpos [n_charges][3]  dE_sol/dy_k in kcal/mol/A (the force is minus it),
 *   dE_dq   [n_charges]     dE_sol/dq_k in kcal/mol/e_c.
 * E = (1/2) q^T B xi with A xi = b(y) q-linear, so
 *   dE/dq = (1/2)(B xi + C^T lam) scaled, dE/dy_k = q_k grad_y(...) (see the
 * kernel comments).  info->e_solv, iters (forward) and adjoint_iters are set. */
int pb_forces(pb_ctx *ctx, const pb_surface *s, const pb_charges *c, const pb_params *p,
              double *dE_dpos, double *dE_dq, pb_info *info);

/* Batched solves of n_sys independent systems (surfaces[b], charges[b]) with
 * shared parameters, in shared launches: one pair sweep over a work list of
 * (system, target block, source range) items per matvec, GMRES
 * in lockstep with per-system state, masks and convergence tests on the
 * device, one restart cycle captured in a hipGraph and replayed until all
 * systems converge.  Restart residuals are FP64; with PB_FP32_IR the Arnoldi
 * matvecs are FP32 (each cycle is a refinement step).  restart <= 32.
 * precond_leaf > 0 applies the block-diagonal leaf preconditioner per system
 * (left preconditioning, as in pb_solve).
 *   e_solv  [n_sys]                     kcal/mol
 *   dE_dpos [sum_b n_b][3], dE_dq [sum_b n_b] (charges concatenated in
 *           system order) or both NULL: when given, the adjoint solves and
 *           gradient sweeps run as well (same meaning as pb_forces).
 *   info    [n_sys] or NULL; seconds is the wall time of the whole call.
 * Returns PB_OK, PB_NOT_CONVERGED (some system hit max_iter) or an error;
 * error messages name the offending system. */
int pb_solve_batch(pb_ctx *ctx, int32_t n_sys, const pb_surface *surfaces,
                   const pb_charges *charges, const pb_params *p, double *e_solv,
                   double *dE_dpos, double *dE_dq, pb_info *info);

/* Potential inside the molecule (eq. eq_inside) at n_points points [n][3]
 * strictly inside the surface, from a surface solution phi, dphi [n_tri]:
 *   reaction[k] = sum_j [K1(x_k, x_j) dphi_j + K2(x_k, x_j) phi_j] a_j
 *   total[k]    = reaction[k] + S1(x_k)
 * in the units of phi (e_c/A divided by 4 pi; x 4 pi 332.0716 for
 * kcal/mol/e_c).  reaction or total may be NULL. */
int pb_potential(pb_ctx *ctx, const pb_surface *s, const pb_charges *c, const pb_params *p,
                 const double *phi, const double *dphi, int64_t n_points, const double *points,
                 double *reaction, double *total);

/* Coulomb energy of the charges in the solute, (332.0716/2) sum_{k != l}
 * q_k q_l / (eps_in |y_k - y_l|) in kcal/mol: E_free of eq. free_energy is
 * E_sol + e_coul. */
int pb_coulomb_energy(pb_ctx *ctx, const pb_charges *c, const pb_params *p, double *e_coul);

/* ---- device-pointer entry points -------------------------------------- */
/* Same operations; every array argument is device memory laid out as above.
 * Validation of the surface runs on the device. */

int pb_matvec_dev(pb_ctx *ctx, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, const pb_params *p, const double *d_x, double *d_y,
                  int transpose, int precision);

int pb_solve_dev(pb_ctx *ctx, int64_t n_vert, int64_t n_tri, const double *d_vert,
                 const int32_t *d_tri, int64_t n_charges, const double *d_pos,
                 const double *d_q, const pb_params *p, double *d_phi, double *d_dphi,
                 pb_info *info);

int pb_forces_dev(pb_ctx *ctx, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, int64_t n_charges, const double *d_pos,
                  const double *d_q, const pb_params *p, double *d_dE_dpos, double *d_dE_dq,
                  pb_info *info);

/* Step 2 (eq. source_terms) on device arrays: d_b [2 n_tri] receives [S1; S2]. */
int pb_source_dev(pb_ctx *ctx, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, int64_t n_charges, const double *d_pos,
                  const double *d_q, const pb_params *p, double *d_b);

/* Step 5 (eq. solvation_energy) of a device-resident surface solution
 * d_phi, d_dphi [n_tri]; the energy (kcal/mol) is written to the host double
 * *e_solv. */
int pb_energy_dev(pb_ctx *ctx, int64_t n_vert, int64_t n_tri, const double *d_vert,
                  const int32_t *d_tri, int64_t n_charges, const double *d_pos,
                  const double *d_q, const pb_params *p, const double *d_phi,
                  const double *d_dphi, double *e_solv);

/* pb_solve_batch with the arrays of every surfaces[b] and charges[b] (vert,
 * tri, pos, q) in device memory, and the gradients d_dE_dpos [sum_b n_b][3],
 * d_dE_dq [sum_b n_b] (both NULL: energies only) written to device memory.
 * e_solv [n_sys] and info [n_sys] stay host arrays.  Same semantics, errors
 * and results as pb_solve_batch. */
int pb_solve_batch_dev(pb_ctx *ctx, int32_t n_sys, const pb_surface *surfaces,
                       const pb_charges *charges, const pb_params *p, double *e_solv,
                       double *d_dE_dpos, double *d_dE_dq, pb_info *info);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as pb_matvec_dev (y = A x or A^T x, FP64 or FP32 pair arithmetic,
 * device arrays), computed with the per-target sweeps in a fixed device
 * scratch array that the library holds on each GPU from the first pb_create
 * there until the process ends (about 14 MB).  The call allocates nothing;
 * n_tri <= 32768 (PB_ERR_ARG beyond, naming the limit).  Results agree with
 * pb_matvec_dev up to rounding (another summation order).  Every call on one
 * GPU shares that GPU's scratch: calls that overlap in time on one GPU, from
 * any context or thread, race.  Same validation and status codes as
 * pb_matvec_dev. */
int pb_matvec_dev_noalloc(pb_ctx *ctx, int64_t n_vert, int64_t n_tri, const double *d_vert,
                          const int32_t *d_tri, const pb_params *p, const double *d_x,
                          double *d_y, int transpose, int precision);

/* ---- preconditioner hooks (tests) ------------------------------------- */
/* The octree leaves used by the preconditioner for leaf size `leaf` (1..100):
 * perm [n_tri] lists the elements leaf by leaf, leaf_start [n_tri + 1] (only
 * the first *n_leaves + 1 entries are written) the leaf boundaries. */
int pb_precond_leaves(pb_ctx *ctx, const pb_surface *s, int leaf, int32_t *perm,
                      int32_t *leaf_start, int64_t *n_leaves);
/* y = M^-1 x (transpose != 0: M^-T x) for the preconditioner that p->precond_leaf
 * selects; x, y: [2 n_tri]. */
int pb_precond_apply(pb_ctx *ctx, const pb_surface *s, const pb_params *p, const double *x,
                     double *y, int transpose);

/* ---- treecode matvec (Sec. 2.2.3) ----------------------------------------- */
/* y = A x with the pair sums evaluated by the treecode of Sec. 2.2.3 (eq.
 * particle_cluster_form) instead of the direct sum: octree leaves of at most
 * `leaf_size` points (N0), multipole acceptance criterion r_c / R <= theta
 * (0 <= theta < 1), and the Taylor polynomial of order `order` (p, 0..5) of
 * each kernel K1..K4 in the source position about the cluster centre.  The
 * result approximates pb_matvec(..., transpose = 0, PB_FP64); theta = 0
 * reproduces it up to rounding.  FP64 throughout.  p->eps_in, eps_out and
 * kappa are used.  x, y: [2 n_tri] host arrays.  counts (may be NULL), if
 * given, receives {particle-cluster interactions, particle-particle pairs,
 * tree nodes} of this matvec.  The paper's setting is theta = 0.8, p = 3,
 * N0 = 100. */
int pb_matvec_tree(pb_ctx *ctx, const pb_surface *s, const pb_params *p, double theta,
                   int order, int leaf_size, const double *x, double *y, int64_t *counts);
/* pb_solve with every GMRES matvec (Arnoldi steps and true-residual checks)
 * replaced by the treecode matvec above, as the paper's treecode solver does
 * (Sec. 2.2.3); the tree is built once per call.  p->precision must be
 * PB_FP64; p->precond_leaf selects the block-diagonal preconditioner as in
 * pb_solve.  Outputs, units and status codes as pb_solve; E_sol carries the
 * treecode's approximation error. */
int pb_solve_tree(pb_ctx *ctx, const pb_surface *s, const pb_charges *q, const pb_params *p,
                  double theta, int order, int leaf_size, double *phi, double *dphi,
                  pb_info *info);

/* ---- launch configuration and autotuning ------------------------------- */
/* The FP32 pair sweep (the hot loop of PB_FP32_IR solves and of their
 * adjoints) comes in two kinds, selected by `targets_per_thread`:
 *   1 or 2             per-target sweep: that many collocation points per
 *                      thread, the source range split into chunks (forward;
 *                      the transposed sweep of this kind has one target per
 *                      thread);
 *   PB_SWEEP_PAIRWISE  pairwise sweep, forward and transposed: each
 *                      unordered pair (i, j) is evaluated once and feeds both
 *                      row i and row j (the distance, exp(-kappa r) and the
 *                      kernel factors they share are computed once).
 * Either kind sizes one launch to about `target_waves` wavefronts.  0 leaves a
 * value unchanged.  Defaults: PB_SWEEP_PAIRWISE, 131072.  Both kinds give the
 * same matvec up to FP32 rounding; only the summation order differs. */
#define PB_SWEEP_PAIRWISE 8
/* FP32 only: the pairwise sweep with each workgroup holding four target tiles
 * and sweeping them over a run of source tiles for a band of such groups,
 * which keeps its partial-sum records to about T^2 / (2 run) + T^2 / (8 band)
 * for T tiles of 256 points (the pairwise kind writes one per tile pair);
 * target_waves / 64 is the number of work items it aims at. */
#define PB_SWEEP_BANDED 16
int pb_set_sweep_config(pb_ctx *ctx, int targets_per_thread, int target_waves);
int pb_get_sweep_config(pb_ctx *ctx, int *targets_per_thread, int *target_waves);
/* The FP64 pair sweeps (forward and transposed: FP64 solves, refinement
 * residuals, adjoints) come in the same two kinds: 1 = one target per thread,
 * PB_SWEEP_PAIRWISE = each unordered pair once.  0 leaves the kind unchanged.
 * Default: PB_SWEEP_PAIRWISE.  The kinds agree up to FP64 rounding. */
int pb_set_fp64_sweep(pb_ctx *ctx, int kind);
int pb_get_fp64_sweep(pb_ctx *ctx, int *kind);
/* Time every candidate configuration (kind in {PB_SWEEP_PAIRWISE, 1, 2} x
 * target_waves in {8192, 16384, 32768, 65536, 131072, 262144}) on this surface with HIP events
 * and keep the fastest in the context.  best_* may be NULL. */
int pb_autotune(pb_ctx *ctx, const pb_surface *s, const pb_params *p, int *best_tpt,
                int *best_waves);

/* Batched solves (pb_solve_batch): the pairwise work items of the batched
 * sweeps take `tiles` source tiles (of 256 points) each; shorter items spread
 * the uneven systems over more blocks, longer ones reuse each target tile's
 * registers longer.  0 leaves the value unchanged; default 4. */
int pb_set_batch_tiles(pb_ctx *ctx, int tiles);
int pb_get_batch_tiles(pb_ctx *ctx, int *tiles);
/* Autotuner of the batched sweeps: on this batch (validated and laid out as by
 * pb_solve_batch, nothing solved), times the batched FP32 forward sweep over
 * all systems with HIP events, one warm-up and three timed launches per
 * candidate, for the pairwise kind with 2, 4, 8, 16 and 32 source tiles per
 * work item and for the per-target kind, and keeps the fastest in the context:
 * the sweep kind as by pb_set_sweep_config, the tiles as by
 * pb_set_batch_tiles.  best_* may be NULL.  Same errors as pb_solve_batch. */
int pb_autotune_batch(pb_ctx *ctx, int32_t n_sys, const pb_surface *surfaces,
                      const pb_charges *charges, const pb_params *p, int *best_kind,
                      int *best_tiles);

/* ---- device memory ------------------------------------------------------ */
/* Cap on the device memory the context holds as scratch (bytes; 0 = no cap,
 * the default).  A call that would grow the context's buffers past the cap
 * fails with PB_ERR_OOM before allocating, and the context stays usable;
 * buffers already held are kept.  For processes that share a GPU.
 * pb_get_memory_used reports the bytes held now. */
int pb_set_memory_limit(pb_ctx *ctx, int64_t bytes);
int pb_get_memory_used(pb_ctx *ctx, int64_t *bytes);

/* ---- kernel timing hook (benchmarks, profiling) ------------------------ */
/* When enabled, every launch of the kernels below is bracketed by a pair of
 * HIP events recorded on the context's stream; elapsed times are collected
 * when the entry point that launched them returns.  `pairs` accumulates the
 * algorithmic pair count of the launches: N(N-1) for a matvec sweep over N
 * collocation points, N*Nc for the source and charge sweeps. */
#define PB_KERNEL_PAIRS_FP64 0      /* matvec pair sweep, FP64 */
#define PB_KERNEL_PAIRS_FP32 1      /* matvec pair sweep, FP32 */
#define PB_KERNEL_PAIRS_FP64_T 2    /* transpose sweep, FP64 */
#define PB_KERNEL_PAIRS_FP32_T 3    /* transpose sweep, FP32 */
#define PB_KERNEL_SOURCE 4          /* source terms */
#define PB_KERNEL_CHARGE 5          /* reaction potential / solid angle at the charges */
#define PB_KERNEL_TREE 6            /* treecode matvec: cluster moments + tree walk */
#define PB_KERNEL_COUNT 7

int pb_profile_enable(pb_ctx *ctx, int enable);
int pb_profile_reset(pb_ctx *ctx);
/* launches, total_ms, pairs may each be NULL. */
int pb_profile_read(pb_ctx *ctx, int kernel, int64_t *launches, double *total_ms, double *pairs);

/* ---- counter calibration (profiling) ------------------------------------ */
/* One launch of a probe kernel whose operation count is known exactly, on the
 * context's stream; returns once it has finished.  For calibrating hardware
 * counters (rocprofv3's VALU instruction and FLOP counts) against a known
 * workload before reading them on the pair sweeps.  262,144 threads (1,024
 * workgroups of 256) each run 8 independent chains of 1,024 steps:
 *   PB_PROBE_FMA_F32: one FP32 fused multiply-add per step;
 *   PB_PROBE_FMA_F64: one FP64 fused multiply-add per step;
 *   PB_PROBE_EXP_F32: one FP32 hardware exp2 (a transcendental) and one FP32
 *                     fused multiply-add per step.
 * *lane_ops receives the number of steps summed over all lanes (2^31); the
 * chains' set-up and final sum add 8 operations per thread at most.  Errors:
 * PB_ERR_ARG for an unknown kind or NULL arguments. */
#define PB_PROBE_FMA_F32 0
#define PB_PROBE_FMA_F64 1
#define PB_PROBE_EXP_F32 2
int pb_probe_valu(pb_ctx *ctx, int kind, int64_t *lane_ops);

/* ---- the FP64 pair functions (testing) ------------------------------------ */
/* exp_out[k] = exp(-x[k]) and rsqrt_out[k] = 1/sqrt(y[k]), evaluated on the
 * device by the functions the FP64 pair sweeps use for the screened Coulomb
 * kernel e^(-kappa r) / (4 pi r) (Sec. 2.2.1, eq. eq_potential): x = kappa r,
 * y = r^2.  For testing their accuracy against a reference and against a
 * host build of the same code.  Host arrays of n values each (0 <= n <=
 * PB_PAIR_MATH_MAX; n = 0 does nothing), with 0 <= x[k] <= PB_PAIR_MATH_XMAX
 * and PB_PAIR_MATH_YMIN <= y[k] <= PB_PAIR_MATH_YMAX (the sweeps stay far
 * inside: kappa r below 3.5e8 even for their padding points, r^2 within
 * [1e-10, 1e13]).  exp(-x) is within 1.32 ulp for x <= 708, subnormal up to
 * x = 745.2 and 0 beyond; 1/sqrt(y) is within 1 ulp.  Returns once the
 * results are in exp_out and rsqrt_out.
 * Errors: PB_ERR_ARG (n out of range, NULL arrays, an argument outside its
 * domain: nothing is written), PB_ERR_OOM, PB_ERR_HIP. */
#define PB_PAIR_MATH_MAX (1 << 24)
#define PB_PAIR_MATH_XMAX 1e12
#define PB_PAIR_MATH_YMIN 1e-30
#define PB_PAIR_MATH_YMAX 1e30
int pb_eval_pair_math(pb_ctx *ctx, int64_t n, const double *x, const double *y,
                      double *exp_out, double *rsqrt_out);

#ifdef __cplusplus
}
#endif

#endif /* PBSOLVE_H */
