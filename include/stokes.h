/*
 * stokes.h -- C ABI of the MI355X (gfx950) solver for the staggered Stokes
 * problem in periodic voxel geometries, by conjugate gradients on the
 * pressure Schur complement S p = g with S = B A^{-1} B^T and g = B A^{-1} f
 * (Pimanov, Iliev, Oseledets, Muravleva, arXiv 2307.05266, Sec. 1,
 * eqs. coupled_matrix, schur_system, schur_rhs; Sec. 3, Algorithm 1).
 *
 * Conventions (Sec. 2.1-2.3):
 *  - The geometry is an N x N x N voxel image, periodic in every direction,
 *    with the box [0,1]^3 (h = 1/N).  A mask byte is 1 for fluid, 0 for
 *    solid; voxel (i,j,k) sits at flat index i + N*(j + N*k) (x fastest).
 *  - Pressure lives at voxel centres (cell arrays of N^3 doubles).
 *  - Velocity lives on voxel faces: a face array holds 3*N^3 doubles,
 *    component c (0=x,1=y,2=z) at offset c*N^3; entry (c, X) is the velocity
 *    on the lower c-face of voxel X, between X - e_c and X.
 *  - A face is an unknown ("active") when both of its voxels are fluid.  The
 *    velocity on every other face is zero (no-slip, eq. stokes_bc_noslip).
 *  - A is the negative velocity Laplacian with the wall half a voxel from
 *    the face centre (mirrored ghost value); B is the negative divergence
 *    and B^T the gradient.
 *  - The body force is uniform; with unit force along an axis the mean
 *    velocity along that axis is the permeability (eq. darcy_law, L = 1).
 *
 * Components: fluid components that cannot carry flow along the force
 * (no closed path in them winds through the periodic box with a non-zero
 * component along the force) have zero velocity in the exact solution;
 * setup removes them, which leaves the solution elsewhere unchanged.  The
 * pressure of each remaining component is fixed to zero mean (Sec. 2.2).
 *
 * Memory and streams: a context owns all of its device memory from setup to
 * destroy (from hipMalloc, stream-ordered allocation, or the caller's
 * allocator: stokes_setup_with_allocator).  All device work of a context runs on one HIP stream (the
 * default stream unless stokes_set_stream is called).  A context must not be
 * used from two threads at once; distinct contexts are independent.
 *
 * Errors: every call returns a stokes_status.  Negative values are errors;
 * on an error the context is left as it was before the call unless stated.
 */
#ifndef STOKES_H
#define STOKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STOKES_OK = 0,
    STOKES_NOT_CONVERGED = 1,   /* warning: the last iterate is kept and valid */
    STOKES_E_ARG = -1,          /* invalid argument; no device work was done */
    STOKES_E_NOMEM = -2,        /* device or host allocation failed */
    STOKES_E_DEVICE = -3,       /* a HIP call failed */
    STOKES_E_BREAKDOWN = -4,    /* NaN/Inf or a non-positive curvature (d, S d) <= 0 */
    STOKES_E_STATE = -5,        /* call out of order (e.g. permeability before solve) */
    STOKES_E_LIMIT = -6         /* geometry exceeds a documented limit */
} stokes_status;

typedef enum {
    STOKES_UZAWA = 0,           /* identity preconditioner (eq. schur_uzawa_prec) */
    STOKES_SIMPLE = 1           /* B diag(A)^{-1} B^T, applied by an inner PCG solve */
} stokes_precond;

/* Operators for stokes_apply / stokes_apply_device. */
typedef enum {
    STOKES_OP_A = 0,            /* faces -> faces: A u */
    STOKES_OP_B = 1,            /* faces -> cells: B u (negative divergence) */
    STOKES_OP_BT = 2,           /* cells -> faces: B^T p (gradient) */
    STOKES_OP_SHAT = 3,         /* cells -> cells: B diag(A)^{-1} B^T p */
    STOKES_OP_DIAG_A = 4,       /* -> faces: diag(A) on active faces (input ignored) */
    STOKES_OP_DIAG_SHAT = 5,    /* -> cells: diag(B diag(A)^{-1} B^T) (input ignored) */
    STOKES_OP_PROJECT = 6,      /* cells -> cells: remove each component's mean */
    STOKES_OP_S = 7,            /* cells -> cells: B A^{-1} B^T p with an inner solve at eps_A */
    STOKES_OP_MG_SHAT = 8,      /* cells -> cells: one cycle of the SIMPLE-matrix multigrid preconditioner,
                                   as the solves apply it (level 1 visited twice where option "mg_visits"
                                   says so; STOKES_E_LIMIT when the geometry has no hierarchy) */
    STOKES_OP_MG_A = 9          /* faces -> faces: one V-cycle of the multigrid preconditioner of A (same) */
} stokes_op;

/* setup flags */
#define STOKES_KEEP_ALL_COMPONENTS 0x1u  /* do not remove non-conducting components */

/* report flags */
#define STOKES_FLAG_NO_FLOW        0x1u  /* no conducting fluid: k = 0 exactly */
#define STOKES_FLAG_ZERO_RHS       0x2u  /* g = 0: the pressure is zero, no outer iteration */
#define STOKES_FLAG_INNER_MAXIT    0x4u  /* an inner solve stopped at its iteration cap */
#define STOKES_FLAG_MG_TWO_VISITS  0x8u  /* the SIMPLE matrix's multigrid cycle visited level 1 twice */

typedef struct stokes_ctx stokes_ctx;

typedef struct {
    int status;                 /* stokes_status of the solve */
    unsigned flags;             /* STOKES_FLAG_* */
    int outer_iters;            /* S applications inside the outer loop */
    int inner_A_iters;          /* total inner iterations with A (including g) */
    int inner_S_iters;          /* total inner iterations with the SIMPLE matrix */
    int n_components;           /* fluid components of the mask as given */
    int n_components_kept;      /* components that carry flow */
    double k_hat;               /* permeability, non-dimensional (L = 1): k_vox / N^2 */
    double k_vox;               /* permeability in voxel units (h = 1) */
    double mean_u[3];           /* box-mean velocity, voxel units */
    double rel_res;             /* ||r_k|| / ||r_0||, r = g - S p */
    double rel_res_prec;        /* ||z_k|| / ||z_0||, z = preconditioned residual */
    double r0_norm;             /* ||g|| */
    double div_norm;            /* ||B u|| of the returned velocity */
    double cond_est;            /* Lanczos estimate from the CG coefficients */
    double ritz_min, ritz_max;
    double porosity;            /* fluid fraction of the mask as given */
    double porosity_effective;  /* after removing non-conducting components */
    double stv_ratio;           /* surface-to-volume ratio (eq. s-t-v-ration), a fraction */
    double seconds;             /* wall time of the solve */
} stokes_report;

/*
 * stokes_setup -- build a context for one geometry (Sec. 2.1-2.2).
 *   ctx    out: new context; untouched on error.
 *   mask   host pointer to N^3 bytes (1 = fluid, 0 = solid), x fastest;
 *          read during the call only (it is copied).
 *   N      voxels per side, 2 <= N <= 800.
 *   force  host pointer to 3 doubles, the uniform body force (finite, not all 0).
 * Returns STOKES_E_ARG for a bad N, a mask byte other than 0/1, or a bad
 * force; STOKES_E_LIMIT when more than 2048 conducting components remain.
 * A geometry without conducting fluid is valid (its permeability is 0).
 */
stokes_status stokes_setup(stokes_ctx **ctx, const uint8_t *mask, int N, const double force[3]);

/* As stokes_setup, with flags (STOKES_KEEP_ALL_COMPONENTS: keep every fluid
 * component; each then carries its own pressure constant). */
stokes_status stokes_setup_ex(stokes_ctx **ctx, const uint8_t *mask, int N, const double force[3],
                              unsigned flags);

/*
 * stokes_setup_on_stream -- as stokes_setup_ex, with all of the context's
 * device work, including setup, on `stream` (a hipStream_t, not NULL), and its
 * device memory allocated and freed in that stream's order (stream-ordered
 * allocation), so that contexts on different streams never wait on each
 * other's allocations.  The stream must outlive the context.  Used by the
 * request server; any caller that owns a stream may use it.
 */
stokes_status stokes_setup_on_stream(stokes_ctx **ctx, const uint8_t *mask, int N, const double force[3],
                                     unsigned flags, void *stream);

/*
 * Device memory from the caller.  alloc returns `bytes` of device memory
 * usable in the order of `stream` (the context's stream, a hipStream_t; NULL =
 * the default stream), or NULL when it cannot; free takes back a block that
 * alloc returned, with the same size and stream.  user is passed through.
 * Both may be called from stokes_setup_with_allocator, stokes_set_option
 * ("precision" allocates the FP32 vectors on first use) and stokes_destroy,
 * always from the thread making that call.
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, size_t bytes, void *stream, void *user);
    void *user;
} stokes_allocator;

/*
 * stokes_setup_with_allocator -- as stokes_setup_ex, with every device buffer
 * of the context taken from the caller's allocator (e.g. a framework's caching
 * allocator, so that the solver shares one memory pool with the caller) and
 * all of the context's device work on `stream` (NULL = the default stream).
 * The allocator struct is copied; its functions must stay callable until
 * stokes_destroy returns, which waits for the stream before freeing.  Every
 * buffer is cleared on the stream after it is allocated, so reused memory is
 * fine.  STOKES_E_ARG when alloc is NULL or lacks either function;
 * STOKES_E_NOMEM when the allocator returns NULL (everything taken so far is
 * freed again).
 */
stokes_status stokes_setup_with_allocator(stokes_ctx **ctx, const uint8_t *mask, int N, const double force[3],
                                          unsigned flags, void *stream, const stokes_allocator *alloc);

/*
 * stokes_setup_batch -- one context for `nmembers` geometries of the same
 * size N (1 <= nmembers <= 32), the k-th from masks[k] (host pointers, read
 * during the call), with the same force and flags, for callers that solve
 * many small problems at once (the request server).  Every kernel launch of
 * the context then advances all members: the launch's second grid dimension
 * is the member, and each member's buffers sit at a fixed stride from the
 * previous member's in one device allocation (stream-ordered on `stream`
 * when it is not NULL).  Reductions and CG scalars stay per member, and a
 * member that has finished a loop sits out the rest of it, so each member's
 * result is bitwise the same whatever the other members are.
 * stokes_solve runs the mixed-precision solve (option "precision" stays 1)
 * for every member and returns the worst member status (its report is member
 * 0's); stokes_batch_result reads each member's.  The operator test hooks
 * (stokes_apply*) refuse batched contexts with STOKES_E_STATE.
 * Errors as stokes_setup_ex, for any member; STOKES_E_ARG for a bad member
 * count or a NULL mask.
 */
stokes_status stokes_setup_batch(stokes_ctx **ctx, const uint8_t *const *masks, int nmembers, int N,
                                 const double force[3], unsigned flags, void *stream);

/*
 * stokes_batch_result -- member `member` of the last solve of a context made
 * by stokes_setup_batch: its report, and (each may be NULL) its pressure (N^3
 * doubles) and velocity (3 N^3 doubles) copied to host memory.
 * STOKES_E_ARG for a bad member, STOKES_E_STATE before a solve.
 */
stokes_status stokes_batch_result(stokes_ctx *ctx, int member, stokes_report *report, double *p, double *u);

/*
 * stokes_estimate_bytes -- upper bound of the device bytes a context for an
 * N^3 box holds (info[9] after setup, plus the FP32 vectors when precision =
 * 1 is used), with the component arrays at their 2048-component limit.
 * Host-only arithmetic; needs no GPU.  STOKES_E_ARG for a bad N, flags or
 * precision (0 or 1) or a NULL bytes.
 */
stokes_status stokes_estimate_bytes(int N, unsigned flags, int precision, int64_t *bytes);

/*
 * stokes_preprocess -- the host-only part of stokes_setup (Sec. 2.1-2.2,
 * eqs. porosity, s-t-v-ration, surface_area); needs no GPU.
 *   mask, N, force, flags  as for stokes_setup_ex.
 *   counts  out, 6 values: fluid voxels (as given), fluid voxels kept,
 *           surface voxels, components (as given), components kept, 0.
 *   fluid   out, N^3 bytes or NULL: 1 where fluid is kept.
 *   label   out, N^3 int32 or NULL: kept-component id, -1 elsewhere
 *           (components numbered by their lowest voxel index).
 * Returns STOKES_E_ARG as stokes_setup does.
 */
stokes_status stokes_preprocess(const uint8_t *mask, int N, const double force[3], unsigned flags,
                                int64_t counts[6], uint8_t *fluid, int32_t *label);

/* Run the context's device work on this HIP stream (hipStream_t; NULL =
 * the default stream).  The caller keeps ownership of the stream. */
stokes_status stokes_set_stream(stokes_ctx *ctx, void *hip_stream);

/*
 * stokes_set_option -- solver options (Sec. 3.1-3.2 stopping criteria):
 *   "eps_A"       inner relative tolerance for A (default 1e-12)
 *   "eps_S"       inner relative tolerance for the SIMPLE matrix (default 1e-12)
 *   "max_outer"   outer iteration cap (default 5000)
 *   "max_inner"   inner iteration cap per solve (default 100000)
 *   "stop_prec"   0: stop on ||r||/||r0|| (default); 1: on ||z||/||z0||
 *                 (the preconditioned norm of Algorithm 1)
 *   "check_every" inner iterations queued between convergence checks (default 0 = adaptive)
 *   "kernel_timing" n > 0: every n-th iteration of each inner solve is launched
 *                 eagerly with each of its kernels bracketed by HIP events
 *                 (0 = off, the default); see stokes_kernel_timing
 *   "fuse_dir_A", "fuse_dir_S"  1: in the multigrid-preconditioned solves,
 *                 form the new direction inside the stencil kernel (one sweep;
 *                 the direction is double-buffered); 0: a separate pointwise
 *                 direction kernel, then the stencil.  Same results bitwise.
 *                 Defaults: 0 for A, 1 for the SIMPLE matrix.
 *   "mg_pipe"     1 (default): the FP64 multigrid-preconditioned solve with the
 *                 SIMPLE matrix runs its three level-0 sweeps (direction and
 *                 stencil, update and restriction, post-smoothing) with their
 *                 loads issued one z-plane ahead of their use; 0: the plain
 *                 forms.  Same arithmetic point by point, results bitwise the
 *                 same.  FP32 inner solves always use the plain forms.
 *   "progress"    n > 0: one line on stderr every n outer iterations
 *                 (iteration, relative residual, permeability, elapsed
 *                 seconds); 0 = silent (default)
 *   "graphs"      1 (default): each inner solve's iteration (CG kernels and
 *                 V-cycle) is captured once as a HIP graph and replayed; 0:
 *                 launched kernel by kernel.  Results are bitwise the same.
 *                 Any stokes_set_option call drops the captured graphs.
 *   "true_velocity" 1: after the solve, recompute u = A^{-1}(f - B^T p)
 *   "sweep_blocks" number of workgroups a sweep aims for (default 1024)
 *   "mg", "mg_A"  1 (default): precondition the inner CG with the SIMPLE matrix
 *                 (resp. with A) by a geometric multigrid V-cycle, the role the
 *                 paper gives to algebraic multigrid (Sec. 3.2); 0: Jacobi.
 *                 The inner stopping test is the same either way.
 *   "mg_omega", "mg_scale", "mg_scale_A", "mg_coarse_sweeps"  V-cycle
 *                 smoothing weight (0.9), coarse-correction scale for the
 *                 SIMPLE matrix (1.7) and for A (1.5) (below 2 keeps the cycle
 *                 SPD), coarsest-level damped-Jacobi sweeps (8)
 *   "mg_coarse_gs" 1 (default): coarse levels with a side below 64 (and not
 *                 the coarsest) smooth by symmetric red-black Gauss-Seidel
 *                 (red then black going down, black then red going up);
 *                 2: every coarse level but the coarsest; 0: damped Jacobi
 *                 with "mg_omega", like level 0
 *   "mg_level_blocks" workgroups a tiled coarse-level sweep aims for (levels
 *                 with a side of 64 or more; default 1024)
 *   "mg_visits"   visits of level 1 per cycle of the SIMPLE matrix.  Two
 *                 visits: after the first visit's result y_1, a second cycle
 *                 from level 1 down on the residual b_1 - A_1 y_1, its result
 *                 added to y_1 (the cycle stays linear and symmetric, and
 *                 positive definite while the eigenvalues of B_1 A_1 stay below
 *                 2, B_1 being the cycle from level 1 down); only where level 1
 *                 has a side of at least 64, is not the coarsest and runs damped
 *                 Jacobi ("mg_coarse_gs" not 2).  0 (default): two visits on
 *                 plain contexts whose level 1 has a side of at least 128, if a
 *                 power iteration at the first SIMPLE-preconditioned solve (or
 *                 STOKES_OP_MG_SHAT application; 20 products B_1 A_1 x)
 *                 puts the largest eigenvalue below 1.8 -- when it does not and
 *                 "mg_scale_deep" is unset, it retries with the corrections
 *                 below level 1 scaled by 1.3 and keeps that scale if the
 *                 estimate then passes; 1: always one visit (the plain
 *                 V-cycle); 2: two wherever allowed, with no estimate.
 *                 Report flag STOKES_FLAG_MG_TWO_VISITS tells which was used.
 *   "mg_scale_deep" scale of the SIMPLE matrix's coarse corrections into
 *                 levels 2 and below (default 0: "mg_scale")
 *   "precision"   0: FP64 throughout (default); 1: mixed -- inner solves with
 *                 A and with the SIMPLE matrix in FP32 (dot products accumulated
 *                 in FP64), outer flexible CG, true residual and permeability
 *                 in FP64, defect-correction cycles with the velocity refined
 *                 in FP64 (the paper's remarks on inexact inner solves, Sec. 3.2)
 *   "eps_A32", "eps_S32"  FP32 inner tolerances of the mixed path (default 1e-5)
 *   "cycle_rtol"  residual reduction per defect-correction cycle (default 1e-4)
 *   "eps_refine"  relative residual of the FP64 velocity refinement (default 1e-12)
 * Unknown keys or out-of-range values give STOKES_E_ARG.
 */
stokes_status stokes_set_option(stokes_ctx *ctx, const char *key, double value);

/*
 * stokes_solve -- CG on S p = g (Algorithm 1, with r = g - S p), starting
 * from p = 0, with the chosen preconditioner, until the relative residual
 * (see "stop_prec") is below tol.  report may be NULL.
 * Returns STOKES_OK, STOKES_NOT_CONVERGED (iteration cap; last iterate kept),
 * STOKES_E_BREAKDOWN, STOKES_E_ARG (tol not positive and finite).
 */
stokes_status stokes_solve(stokes_ctx *ctx, stokes_precond precond, double tol, stokes_report *report);

/*
 * stokes_solve_rhs -- CG on S p = g for a given right-hand side (the
 * Schur-complement system of Sec. 1, eq. schur_system, with g from the caller
 * instead of g = B A^{-1} f): g is a host array of N^3 doubles, read on the
 * fluid cells during the call, and must lie in the range of B (e.g. g = B xi,
 * which makes it sum to zero over every component).  Starts from p = 0 and
 * u = 0, so the returned velocity is -A^{-1} B^T p and the report's
 * permeability fields refer to it.  Only an exactly zero g skips the loop.
 * FP64 plain contexts only: STOKES_E_STATE for a batched context or with
 * "precision" 1; otherwise as stokes_solve.
 */
stokes_status stokes_solve_rhs(stokes_ctx *ctx, stokes_precond precond, double tol, const double *g,
                               stokes_report *report);

/* Permeability of the last solve along the force, non-dimensional (Sec. 2.3):
 * k_hat = <u . f> / |f|^2 / N^2.  STOKES_E_STATE before a solve. */
stokes_status stokes_permeability(stokes_ctx *ctx, double *k_hat);

/* Report of the last solve (STOKES_E_STATE before a solve). */
stokes_status stokes_get_report(stokes_ctx *ctx, stokes_report *report);

/* Per outer iteration k = 1..n of the last solve, 8 doubles each:
 * ||r_k||/||r_0||, ||z_k||/||z_0||, k_hat(u_k), inner A iters, inner S iters,
 * alpha_{k-1}, beta_{k-1} (0 if the loop stopped first), 0.
 * Writes min(n, cap) rows to out (host), returns n in *n_out. */
stokes_status stokes_history(stokes_ctx *ctx, double *out, int cap, int *n_out);

/* Copy the last solution to host memory: p (N^3, zero-mean per component,
 * 0 in solid) and u (3*N^3, 0 on inactive faces).  Either may be NULL. */
stokes_status stokes_get_fields(stokes_ctx *ctx, double *p, double *u);

/* Apply one operator (stokes_op) to a host field, writing a host field.
 * Entries of `in` on inactive faces / solid cells are treated as 0.
 * Sizes: faces 3*N^3 doubles, cells N^3 doubles. */
stokes_status stokes_apply(stokes_ctx *ctx, int op, const double *in, double *out);

/* As stokes_apply, with device pointers; runs on the context's stream and
 * returns without waiting for it. */
stokes_status stokes_apply_device(stokes_ctx *ctx, int op, const double *in, double *out);

/*
 * stokes_apply_device_noalloc -- for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  As stokes_apply_device, with the same kernels and the
 * same results bitwise, but the masked copy of the input and the partial sums
 * of the projection live in a fixed 32 MiB device array of the library (one
 * copy per GPU, held until the process ends; its address is resolved when a
 * context is set up on that GPU) instead of the context's work vectors, and
 * the result goes straight to `out`.  The call allocates nothing and issues
 * only device-to-device copies and kernel launches on the context's stream;
 * it returns without waiting.
 *   op       STOKES_OP_A, _B, _BT, _SHAT, _DIAG_A, _DIAG_SHAT or _PROJECT;
 *            the inner-solve and V-cycle operators (STOKES_OP_S, _MG_SHAT,
 *            _MG_A) need the context's work vectors: STOKES_E_ARG.
 *   in, out  device pointers, sizes as for stokes_apply (in is ignored by the
 *            DIAG operators; in == out is allowed for STOKES_OP_PROJECT only,
 *            otherwise the two must not overlap).
 * Limit: the input copy (3 N^3 doubles for A and B, N^3 for B^T and the
 * SIMPLE matrix; none for PROJECT and the DIAG operators) plus the partial
 * sums (at most 4096 doubles, or 257 K for K > 1 components) must fit in
 * 32 MiB, i.e. N <= 111 for A and B, N <= 161 for B^T and SHAT; beyond it
 * the call returns STOKES_E_LIMIT and does no device work.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap in time on one GPU (several streams or threads)
 * race, and the caller must order them (e.g. one stream).
 */
stokes_status stokes_apply_device_noalloc(stokes_ctx *ctx, int op, const double *in, double *out);

/* info[0..11]: N, fluid voxels (as given), fluid voxels kept, surface voxels,
 * components (as given), components kept, active x/y/z faces (3 values),
 * device bytes held, coarse levels of the multigrid hierarchy for the SIMPLE
 * matrix and for A (0: none -- odd N, or the coarsest level would not fit one
 * workgroup -- and that inner solve uses Jacobi-PCG). */
stokes_status stokes_info(stokes_ctx *ctx, int64_t info[12]);

/* Device time of the inner-loop kernels since the last call for that kernel,
 * measured with HIP events around the sampled launches (see "kernel_timing")
 * on the context's stream.  kernel: 0 = A direction, 1 = A stencil,
 * 2 = A update, 3 = SIMPLE direction, 4 = SIMPLE stencil, 5 = SIMPLE update,
 * and the voxel-level multigrid kernels: 6 = A restriction, 7 = A smoothing,
 * 8 = SIMPLE restriction, 9 = SIMPLE smoothing, 10 = A update fused with the
 * restriction, 11 = SIMPLE update fused with the restriction, 12 = A
 * direction fused with the stencil, 13 = SIMPLE direction fused with the
 * stencil (10..13: the multigrid-preconditioned solves), and the FP64 SIMPLE
 * solve's software-pipelined forms ("mg_pipe"): 14 = update fused with the
 * restriction, 15 = smoothing, 16 = direction fused with the stencil.  Returns the total
 * milliseconds and the number of timed launches (launches queued after
 * convergence return at once and are counted too), and the algorithmic bytes one launch
 * moves (each input read once, each output written once, in FP64). */
stokes_status stokes_kernel_timing(stokes_ctx *ctx, int kernel, double *ms_total, int64_t *launches,
                                   double *bytes_per_launch);

/* Free everything the context holds.  NULL is ignored. */
void stokes_destroy(stokes_ctx *ctx);

/* Static string naming a status. */
const char *stokes_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* STOKES_H */
