/*
 * cps.h -- C-ABI of the MI355X (gfx950) compact immersed-interface Poisson solver.
 *
 * The library solves the 3D Dirichlet Poisson problem of Hosseinverdi & Fasel (arXiv
 * 1901.08269), Eq. (poisson):
 *     Laplacian u = f  in the fluid region (level set phi > 0),
 *     u = g            on the box walls and on the interface Gamma (phi = 0),
 *     u = 0            inside the bodies (phi <= 0),
 * The fluid region may also be the inside of a closed interface (the interior problem of
 * Sec. 4, Problem 4): wall nodes may then lie in phi <= 0, provided no fluid node is among
 * their neighbours (no row of the scheme reaches them; they keep the value g).
 * on a tensor-product nonuniform grid (Sec. 2), with the fourth-order compact 27-point
 * scheme (Sec. 2.1, Eqs. A27/As_qs/q), modified at irregular points next to Gamma
 * (Secs. 2.2-2.3, Eqs. A27_mod/bc/cor and their multiple-intersection forms), and solves
 * the resulting system B u = q + b (Sec. 3, Eq. Bu=q, split B = A-bar + C of Eq. Bdec)
 * by right-preconditioned BiCGSTAB (Sec. 3.2, Alg. 1) whose preconditioner is the
 * second-order 7-point operator K with Shortley-Weller rows at Gamma (Sec. 3.3, Eqs.
 * A7/A7_mod), solved approximately by a fixed linear inner solver: one multigrid V-cycle
 * (default), a fixed number of Chebyshev-Jacobi steps, or a fixed number of iterations of
 * the strongly implicit procedure (cps_options.precond).
 *
 * Conventions shared by every entry point
 *   - Grid: nx, ny, nz points per direction INCLUDING both wall planes; coordinates
 *     x[nx], y[ny], z[nz] strictly increasing.  Unknowns are the interior nodes with
 *     phi > 0: (nx-2)(ny-2)(nz-2) minus the solid nodes (Sec. 3, first paragraph).
 *   - Node arrays have nx*ny*nz float64 entries, node (i,j,k) at index i + nx*(j + ny*k),
 *     0-based, x fastest.
 *   - Pointers are host pointers unless cps_options.device_ptrs = 1, in which case every
 *     array argument of every call on that solver is a device pointer (e.g. a torch
 *     tensor's data_ptr()).  The caller owns all input and output buffers; the library
 *     copies what it needs and never keeps a caller pointer after a call returns.
 *   - Work is ordered on cps_options.stream (NULL = the null stream); every call
 *     synchronises that stream before it returns.  A solver object is not thread-safe.
 *   - Return value: 0 on success or a negative CPS_E* code; cps_strerror names it.
 */
#ifndef CPS_H
#define CPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPS_OK 0
#define CPS_EINVAL (-1)      /* bad sizes, non-increasing coordinates, NaN/Inf input, bad option */
#define CPS_EGEOM (-2)       /* a wall node inside a body (phi <= 0) has a fluid neighbour, or a
                              * modified line is singular */
#define CPS_ENOMEM (-3)      /* device or host allocation failed */
#define CPS_EDEVICE (-4)     /* a HIP runtime call failed or no device is present */
#define CPS_EBREAKDOWN (-5)  /* BiCGSTAB broke down more often than max_restarts allows */
#define CPS_ENOCONV (-6)     /* max_iters reached (CPS_MIXED with fp64_finish 0: also a stagnating
                              * or max_refine-long refinement); u holds the last iterate, stats
                              * are filled */
#define CPS_ENAN (-7)        /* the iteration produced NaN/Inf */

#define CPS_FP64 0           /* plain mode: every sweep in FP64 */
#define CPS_MIXED 1          /* FP32 inner BiCGSTAB inside an FP64 iterative-refinement loop */

#define CPS_PRECOND_CHEBYSHEV 0  /* inner_iters Chebyshev-Jacobi steps on K per apply */
#define CPS_PRECOND_MULTIGRID 1  /* one multigrid V-cycle on K per apply */
#define CPS_PRECOND_SIP 2        /* sip_iters iterations of the strongly implicit procedure on K */

typedef struct cps_solver cps_solver; /* opaque; owns all of its device memory */

typedef struct cps_options {
    int32_t struct_size;   /* = sizeof(cps_options) */
    int32_t precision;     /* CPS_FP64 or CPS_MIXED */
    int32_t inner_iters;   /* Chebyshev-Jacobi steps per preconditioner apply (default 24; the
                            * paper's MSI preconditioner runs 8 inner iterations, Sec. 4) */
    int32_t max_iters;     /* cap on BiCGSTAB iterations (summed over refinement steps) */
    int32_t max_refine;    /* CPS_MIXED: cap on FP32 refinement steps (see fp64_finish) */
    int32_t max_restarts;  /* restarts after breakdown or a failed true-residual check */
    int32_t device_ptrs;   /* 1: array arguments are device pointers */
    int32_t kernel_timing; /* n > 0: time the preconditioner's Chebyshev sweeps on the problem's
                            * grid (multigrid: every smoothing step there but the pointwise first
                            * step of a pre-smoothing pass; Chebyshev: steps 1 .. inner_iters - 1)
                            * in every n-th preconditioner apply, each by a pair of HIP events that
                            * its launch stamps with the kernel's start and end (stats); sweeps
                            * queued after convergence are left out; 0: off */
    double inner_tol;      /* CPS_MIXED: residual reduction asked of each FP32 inner solve */
    double lam_lo, lam_hi; /* Chebyshev interval for the spectrum of diag(K)^-1 K (default
                            * hi = 2; lo = 0 selects max(hi / (4 inner_iters^2), lambda_1) with
                            * lambda_1 = (1/3) sum_d (1 - cos(pi / (n_d - 1)))) */
    void *stream;          /* hipStream_t the library launches on; NULL = null stream */
    /* How K phi = rho is solved approximately inside the preconditioner (Sec. 3.3 leaves the
     * inner solver open).  CPS_PRECOND_MULTIGRID: one V-cycle.  A coarser grid keeps the
     * even-indexed points and the last point along every axis (while every axis has at least
     * 17 points and the grid has more than 4096 interior points); its K is built from the
     * level set at its nodes.  Prolongation is trilinear
     * interpolation in the physical coordinates; restriction is its transpose with each row
     * divided by its sum.  Smoother: mg_nu Chebyshev-Jacobi steps before and after each
     * coarse correction on [mg_smooth_lo, lam_hi]; the coarsest grid takes mg_coarse_steps
     * steps on [lambda_1, lam_hi] of that grid.  The cycle is a fixed linear map of rho. */
    int32_t precond;         /* CPS_PRECOND_MULTIGRID (default) or CPS_PRECOND_CHEBYSHEV */
    int32_t mg_levels;       /* most levels, this grid included, 1..16 (default 16) */
    int32_t mg_nu;           /* smoothing steps before and after, 1..64 (default 2) */
    int32_t mg_coarse_steps; /* steps on the coarsest grid, 1..64 (default 8) */
    double mg_smooth_lo;     /* lower end of the smoother's interval, in (0, lam_hi) (default 0.2) */
    /* CPS_PRECOND_SIP: the strongly implicit procedure (Stone's partial-cancellation incomplete
     * factorisation of K, L U with unit upper diagonal, unknowns in x-fastest order; the
     * unknowns one factor entry beyond K's stencil reaches are approximated by sip_alpha x
     * (the two stencil neighbours it lies between minus the centre); sip_alpha = 0 is the
     * incomplete factorisation without fill), sip_iters iterations from phi = 0 per apply
     * (the paper runs 8 inner iterations of its modified strongly implicit procedure,
     * Sec. 4).  The substitutions run hyperplane by hyperplane (i + j + k = const), one
     * launch each: far slower on a GPU than the parallel inner solvers. */
    int32_t sip_iters;       /* 1..64 (default 8) */
    int32_t fp64_finish;     /* CPS_MIXED, 1 (default): when a refinement step reduces
                              * ||D^-1 r||_2 by less than sqrt(2) (the FP32 solve no longer
                              * resolves the correction), or max_refine steps or max_restarts
                              * restarts are spent, continue with FP64 BiCGSTAB from the
                              * current iterate (stats: iters - iters_fp32 FP64 iterations);
                              * 0: return CPS_ENOCONV / CPS_EBREAKDOWN there */
    double sip_alpha;        /* in [0, 1] (default 0.9) */
} cps_options;

typedef struct cps_stats {
    int32_t struct_size;    /* = sizeof(cps_stats) */
    int32_t iters;          /* BiCGSTAB iterations (all precisions) */
    int32_t iters_fp32;     /* of which FP32 inner iterations (CPS_MIXED) */
    int32_t refine_steps;
    int32_t restarts;
    int32_t status;         /* return code of the solve */
    int64_t n_unknowns, n_irregular, n_solid, nnz_irregular, fallback_lines;
    double rel_residual;        /* ||b - B u||_2 / ||b||_2 over unknowns, FP64, paper row scaling */
    double rel_residual_jacobi; /* ||D^-1 (b - B u)||_2 / ||D^-1 b||_2, D = diag(B) */
    double min_ibi_frac;        /* min over IBIs of |x_fluid - x_IBI| / segment length */
    double setup_ms, solve_ms;
    double sweep_ms;            /* kernel_timing: summed execution time of the timed sweeps
                                 * (kernel start to end; no launch gaps) */
    int64_t sweep_launches;     /* kernel_timing: number of sweeps in them */
    int64_t sweep_points;       /* interior points one sweep processes */
    double sweep_bytes;         /* kernel_timing: algorithmic bytes the timed sweeps move (every
                                 * vector a sweep reads or writes, once per interior point: three
                                 * for the first step of a pass, four for the others) */
    double sweep_full_ms;       /* kernel_timing: the part of sweep_ms spent in full-traffic
                                 * sweeps (those that read an x_{k-1}: four vectors) */
    int64_t sweep_full_launches;
    double warm_alpha;          /* warm start: the factor it was scaled by -- 1 if its residual is
                                 * at most ||b||_2, else argmin over alpha of ||b - alpha B u0||_2
                                 * (0 rejects it); 0 without a warm start */
} cps_stats;

/* Fill `o` with the defaults: CPS_FP64, 24 inner iterations, max_iters 20000,
 * max_refine 40, max_restarts 5, host pointers, inner_tol 1e-4, the default Chebyshev
 * interval, null stream, no kernel timing, the multigrid preconditioner (up to 16 levels,
 * 2 + 2 smoothing steps on [0.2, lam_hi], 8 coarsest-grid steps), 8 strongly implicit
 * iterations with alpha 0.9 when that preconditioner is chosen. */
void cps_default_options(cps_options *o);

/* Build the discrete problem (Secs. 2-3): classify nodes from the sign of phi (Sec. 2,
 * Fig. grid_point_types), locate the interface intersections (IBIs) on grid segments where
 * phi changes sign (degree-5 interpolation of nodal phi; g at an IBI from the same
 * interpolation of nodal g), build the modified rows of B at irregular nodes and the
 * Shortley-Weller rows of K, and assemble the right-hand side q + b (Eqs. q, bc, cor).
 * phi, g, f: nx*ny*nz float64 node arrays.  g must be a smooth field whose values at wall
 * nodes and at the IBIs are the Dirichlet data; f is read at fluid and wall nodes.
 * opt may be NULL (defaults).  On success *out receives a new solver. */
int cps_setup(cps_solver **out, int32_t nx, int32_t ny, int32_t nz, const double *x, const double *y,
              const double *z, const double *phi, const double *g, const double *f, const cps_options *opt);

/* Replace f and g (same grid and geometry) and rebuild the right-hand side. */
int cps_set_rhs(cps_solver *s, const double *f, const double *g);

/* Solve B u = q + b (Alg. 1) until ||r||/||b|| <= tol and ||D^-1 r||/||D^-1 b|| <= tol in
 * FP64.  u: nx*ny*nz float64; if warm_start is nonzero its unknown entries are the initial
 * guess (NaN/Inf there -> the guess is discarded and 0 used), else the guess is 0.  On
 * return u holds the solution at unknowns, g at wall nodes and 0 at solid nodes.  st may
 * be NULL.  CPS_MIXED: FP32 BiCGSTAB solves of the correction equation inside FP64
 * iterative refinement, finished in FP64 if they stagnate (cps_options.fp64_finish).
 * Returns CPS_OK, CPS_ENOCONV, CPS_EBREAKDOWN or CPS_ENAN (u then holds the last finite
 * iterate). */
int cps_solve(cps_solver *s, double tol, double *u, int32_t warm_start, cps_stats *st);

/* Residual history of the last cps_solve on s (Alg. 1's recursive residual).
 * iter_res[q], q < *n_iter (= stats.iters): ||D^-1 r||_2 / ||D^-1 b||_2 (D = diag B) of the
 * recursive residual r after the solve's (q+1)-th BiCGSTAB iteration, in the order run; in
 * CPS_MIXED the FP32 iterations' r is that of the correction equation, which estimates the
 * FP64 residual of the corrected solution.  true_res[2q], true_res[2q+1], q < *n_true: the
 * FP64 true residual ||b - B u||_2 / ||b||_2 and ||D^-1 (b - B u)||_2 / ||D^-1 b||_2 before
 * each restart pass or refinement step, and at the end (the last pair is the final
 * residual).  At most cap_iter values and cap_true pairs are copied (host pointers; an array
 * may be NULL when its cap is 0); *n_iter and *n_true (either may be NULL) receive the full
 * lengths.  CPS_EINVAL for a negative cap or a NULL array with a positive cap. */
int cps_get_history(cps_solver *s, double *iter_res, int32_t cap_iter, int32_t *n_iter, double *true_res,
                    int32_t cap_true, int32_t *n_true);

/* r = b - B u at unknown nodes (0 elsewhere), FP64, using the unknown entries of u.
 * r may be NULL.  rel[0] = ||r||_2/||b||_2, rel[1] = ||D^-1 r||_2/||D^-1 b||_2 (rel may be NULL). */
int cps_residual(cps_solver *s, const double *u, double *r, double *rel);

/* y = B x (Eq. Bu=q, B = A-bar + C of Eq. Bdec) at unknown nodes, 0 elsewhere.
 * precision CPS_FP64 applies the FP64 operator, CPS_MIXED the FP32 operator (x rounded to
 * FP32 first, y widened back).  Entries of x at non-unknown nodes are ignored. */
int cps_apply(cps_solver *s, const double *x, double *y, int32_t precision);

/* phi = M rho: the preconditioner of Alg. 1 (applied to p and to s): an approximate solve of
 * K phi = rho (Sec. 3.3) from phi = 0 -- inner_iters Chebyshev-Jacobi steps, one multigrid
 * V-cycle, or sip_iters strongly implicit iterations (cps_options.precond); FP64 or FP32 as
 * above. */
int cps_precond(cps_solver *s, const double *rho, double *phi, int32_t precision);

/* Copy out the right-hand side q + b (node array, 0 at non-unknowns) and the node types
 * (int8 node array: 0 wall, 1 regular fluid, 2 irregular fluid, 3 solid).  Either may be NULL. */
int cps_get_rhs(cps_solver *s, double *rhs, int8_t *types);

/* Sizes: out[0] unknowns, [1] irregular rows, [2] solid nodes, [3] stored nonzeros of the
 * irregular rows, [4] fallback lines, [5] nx*ny*nz. */
int cps_get_info(cps_solver *s, int64_t out[6]);

/* Export the irregular rows (Eqs. A27_mod, bc, cor): node[n_irr] (int64 node index, rows in
 * increasing node order), ptr[n_irr+1], col[nnz] (int64 node index of an unknown), val[nnz]
 * (FP64 coefficient of B), krow[7*n_irr] (K row: diag, -x, +x, -y, +y, -z, +z).  Host
 * pointers always; any may be NULL. */
int cps_get_irregular(cps_solver *s, int64_t *node, int64_t *ptr, int64_t *col, double *val, double *krow);

void cps_destroy(cps_solver *s);
const char *cps_strerror(int code);

/* ---------------------------------------------------------------------------------------
 * Learned warm start: a 4-level 3D convolutional encoder-decoder on the grid coarsened 4x
 * per direction (inputs: cell means of f, phi, g; output: the cell means of u), trained
 * on solutions of this solver.  It only supplies the initial guess of cps_solve; the
 * BiCGSTAB solve always runs to the requested tolerance from it.
 * Network arrays are always DEVICE pointers (FP32): inputs [batch][in_ch][nc^3], targets,
 * masks and predictions [batch][nc^3], index (x + nc (y + nc z)) inside a sample.
 * Parameters: FP32, flat, per 3x3x3 layer W[co][ci][kz][ky][kx] then b[co] in the order
 * E0a E0b E1a E1b E2a E2b E3a E3b D2a D2b D1a D1b D0a D0b, then the 1x1x1 head (c0
 * weights, 1 bias).  Host pointers for cps_model_set_params / get_params.
 * ------------------------------------------------------------------------------------- */
typedef struct cps_model cps_model;   /* opaque; owns weights, Adam state and activations */

typedef struct cps_model_spec {
    int32_t struct_size;  /* = sizeof(cps_model_spec) */
    int32_t nc;           /* coarse points per direction (multiple of 8) */
    int32_t batch;        /* largest batch the model is sized for */
    int32_t in_ch;        /* input channels (3: f, phi, g) */
    int32_t channels[4];  /* per level, multiples of 16 in [16, 64]; channels[0] = 16 */
    uint64_t seed;        /* initialisation seed */
} cps_model_spec;

int64_t cps_model_param_count(const cps_model_spec *spec);
/* stream: hipStream_t for all work of this model (NULL = null stream) */
int cps_model_create(cps_model **m, const cps_model_spec *spec, void *stream);
int cps_model_set_params(cps_model *m, const float *params, int64_t n);          /* resets Adam */
int cps_model_get_params(cps_model *m, float *params, float *grads, int64_t n);  /* grads: last step */
/* pred = network(inputs) */
int cps_model_forward(cps_model *m, const float *inputs, int32_t batch, float *pred);
/* forward + masked mean-squared error + backward (+ one Adam step with learning rate lr
 * when update != 0).  mask may be NULL (all ones).  *loss_out = loss before the update. */
int cps_model_train_step(cps_model *m, const float *inputs, const float *target, const float *mask, int32_t batch,
                         float lr, int32_t update, double *loss_out);
/* Network input of one problem: cell means over 4^3 blocks of interior nodes of f, phi, g
 * (scaled: sigma = RMS over nodes of sqrt(g^2 + (f / 3 pi^2)^2)); with u non-NULL also the
 * target: cell means over the same blocks of u / sigma, with g in place of u at nodes inside
 * a body (phi <= 0), i.e. of the solution's continuation by g.  The solver grid must have 4 nc interior points per
 * direction.  u, inputs, target: device pointers; sigma: host (may be NULL). */
int cps_model_restrict(cps_model *m, cps_solver *s, const double *u, float *inputs, float *target, double *sigma);
/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): cps_model_restrict with the same arguments, results
 * and errors, that calls no allocating routine.  Its scratch (the 256 per-block partial sums of
 * the sigma reduction and sigma itself: 257 doubles, 2 KiB) is a fixed device array of the
 * library, one per device, kept until the process ends; the reduction uses 256 blocks at every
 * grid size, so no size exceeds it.  Every call on a device shares that array: calls that
 * overlap on one device (other streams, other threads) race and must be serialised by the
 * caller.  The first call on a device looks up the array's address there; later calls only
 * launch kernels, copy sigma out and synchronise the model's stream. */
int cps_model_restrict_noalloc(cps_model *m, cps_solver *s, const double *u, float *inputs, float *target,
                               double *sigma);
/* u0 (device, nx*ny*nz FP64) = sigma * trilinear prolongation of the network's prediction
 * for the solver's problem; pass it to cps_solve as the warm start. */
int cps_model_predict(cps_model *m, cps_solver *s, double *u0);
/* The same warm start from the fields themselves, without a solver, queued on `stream` (NULL:
 * the model's stream) and returned from at once, so that it can run beside the solver's setup
 * of the same problem.  phi, g, f: device FP64 arrays of the nx x ny x nz grid (x fastest; the
 * grid must have 4 nc interior points per direction), ready on `stream` when it reaches the
 * call (order their producer before it); u0: device, nx*ny*nz FP64, every node written,
 * complete when `stream` passes the call.  The call uses the model's work buffers: calls on
 * one model must not overlap.  CPS_EINVAL for a NULL pointer or a grid of another size. */
int cps_model_predict_fields(cps_model *m, int32_t nx, int32_t ny, int32_t nz, const double *phi, const double *g,
                             const double *f, double *u0, void *stream);
/* Write the weights to `path` (raw binary: magic "CPSNET01", the spec, the parameter count,
 * the FP32 weights).  CPS_EINVAL if the file cannot be written. */
int cps_model_save(cps_model *m, const char *path);
/* A training checkpoint: the weights plus the optimiser's state -- Adam's step count and its
 * two FP32 moment vectors (magic "CPSNET02") -- so that cps_model_train_step continues after
 * cps_model_load exactly as it would have without the interruption. */
int cps_model_save_checkpoint(cps_model *m, const char *path);
/* Read either file into m (whose spec must have the same parameter count).  Weights only:
 * Adam starts afresh (zero moments, step 0); a checkpoint restores its state too.
 * CPS_EINVAL for a missing, short or foreign file. */
int cps_model_load(cps_model *m, const char *path);
void cps_model_destroy(cps_model *m);

#ifdef __cplusplus
}
#endif
#endif /* CPS_H */
