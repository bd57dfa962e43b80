/*
 * kct.h -- C ABI of the Krylov cone-beam CT library for MI355X (gfx950).
 *
 * The library solves the CBCT problem A x + e = b (paper Sec. 1, eq.
 * (original_pbm)) with the Krylov methods of Sec. 2 using only products with
 * the matched pair A (cone-beam forward projection) and A^T (its exact
 * transpose), both hand-written HIP kernels.
 *
 * System matrix.  Row i is the ray from the source to the centre of detector
 * pixel i; column j is voxel j; a_ij is the length in mm of ray i inside
 * voxel j (Siddon's radiological path; the paper leaves the discretisation to
 * its toolbox).  A is never stored.
 *
 * Geometry (the paper gives none; the convention is fixed here):
 *   voxel (i,j,k) = half-open box [X0+i vx, X0+(i+1) vx) x [Y0+j vy, ...) x
 *                   [Z0+k vz, ...), X0 = ox - nx vx/2 (same for y, z);
 *   source        s = (DSO cos t, DSO sin t, 0) for gantry angle t;
 *   detector      centre s + DSD (-cos t, -sin t, 0), axes
 *                 e_u = (-sin t, cos t, 0) and e_v = (0, 0, 1);
 *   pixel (iu,iv) centre = centre + (iu-(nu-1)/2) du e_u + (iv-(nv-1)/2) dv e_v.
 * Lengths are in mm, angles in radians, attenuation in 1/mm.
 *
 * Layouts.  Volumes are contiguous [nz][ny][nx] (x fastest); projections are
 * contiguous [n_angles][nv][nu] (u fastest).
 *
 * Ownership.  The caller allocates and owns every device buffer passed in
 * (volumes, projections, right-hand side, solution, workspace, history).  A
 * plan owns its geometry tables, the back projector's partial volumes for
 * small volumes (allocated with the plan) and, after kct_plan_reserve, the
 * padded volume copies that plain kct_forward calls read;
 * kct_plan_device_bytes reports that memory.  The library never frees caller
 * memory.  Only kct_plan_create, kct_plan_reserve and kct_plan_destroy
 * allocate or free device memory; no other call does.
 *
 * Streams.  Every call that takes a `stream` (a hipStream_t, or NULL for the
 * null stream) only enqueues work on it and returns; the caller synchronises.
 * kct_forward and kct_backproject calls on one plan share the plan's scratch
 * (the padded volume copies; for small volumes, the back projector's partial
 * volumes), so they must not overlap in time (use one plan per stream for
 * that).  Solves keep that scratch in their own workspace and only read the
 * plan, so solves on one plan may run concurrently on different streams.
 *
 * Errors.  Argument and geometry checks happen before anything is enqueued and
 * return a status; kct_last_error() then holds a message for the calling
 * thread.  No C++ exception crosses this interface and the library never
 * aborts.  A launch failure returns KCT_E_DEVICE.  Krylov breakdown (a zero
 * norm, e.g. b = 0) is not an error: the remaining iterations leave x
 * unchanged and report it in the history.  The back projector sizes its
 * per-tile detector patch and per-voxel column count from bounds the plan
 * derives from the geometry's extreme magnification; a footprint beyond them
 * is not expected for any geometry the plan accepts, but if one occurs the
 * sums are truncated and the library says so: kct_plan_check returns
 * KCT_E_GEOMETRY, and a solve records done code 4 in its history.
 */
#ifndef KCT_H
#define KCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kct_status {
    KCT_OK = 0,
    KCT_E_INVALID_ARG = 1, /* null pointer, bad size or unknown enum value          */
    KCT_E_GEOMETRY = 2,    /* geometry that the convention above cannot represent   */
    KCT_E_DTYPE = 3,       /* storage type not supported for this call              */
    KCT_E_OOM = 4,         /* device allocation by the library failed               */
    KCT_E_BUDGET = 5,      /* a caller-provided buffer is too small                 */
    KCT_E_DEVICE = 6,      /* a HIP call or kernel launch failed                    */
    KCT_E_NONFINITE = 7,   /* reserved: a solver that meets a NaN or Inf reports it
                              in history column 3 (the host never waits on it)    */
    KCT_E_STATE = 8        /* reserved                                              */
} kct_status;

/* Storage types of device vectors.  Arithmetic is FP32 for ray and voxel
 * accumulation and FP64 for the Krylov scalars, whatever the storage type. */
typedef enum kct_dtype {
    KCT_F32 = 0,
    KCT_BF16 = 1, /* bfloat16, round-to-nearest-even on store */
    KCT_F16 = 2   /* IEEE binary16, round-to-nearest-even on store */
} kct_dtype;

/* Circular cone-beam geometry (see the convention at the top of this file). */
typedef struct kct_geometry {
    int32_t nx, ny, nz;    /* voxels per axis, > 0                                   */
    double vx, vy, vz;     /* voxel size (mm), > 0                                    */
    double ox, oy, oz;     /* volume centre offset from the rotation axis (mm)        */
    int32_t nu, nv;        /* detector pixels along e_u and e_v, > 0                  */
    double du, dv;         /* pixel pitch (mm), > 0                                   */
    double dso, dsd;       /* source-origin and source-detector distances (mm)        */
    int32_t n_angles;      /* number of gantry angles, > 0                            */
    const double *angles;  /* host pointer to n_angles radians; copied by the plan    */
} kct_geometry;

typedef struct kct_plan kct_plan;

/*
 * Create a plan for `geom` on HIP device `device`: validates the geometry
 * (DSO > 0, DSD > DSO, and the volume's bounding cylinder strictly between
 * the source orbit and the detector plane), builds the per-angle FP64 tables
 * on the host (cos/sin evaluated once, in double precision) and copies them
 * to the device.  Returns KCT_E_GEOMETRY for a geometry outside the
 * convention.  `*out` receives the plan, owned by the caller until
 * kct_plan_destroy.
 *
 * The plan also fixes the projectors' launch shapes from the geometry.  For
 * tuning, these environment variables, read here, override the choice
 * (values outside the listed sets are ignored):
 *   KCT_FWD_PREFETCH     0, 1, 2  segments the forward gathers ahead (2 for
 *                                 volumes with 16-bit padded copies, else 1)
 *   KCT_FWD_LANES_U      16, 32, 64  pixels per wave row in the forward
 *                                 (32 when neighbouring rays are a voxel or
 *                                 more apart at the axis, else 16)
 *   KCT_FWD_WAVE_ANGLES  1, 4, 8, 16  angles per forward workgroup, one
 *                                 wave each (8 where the padded copies stay
 *                                 16-bit, else 4)
 *   KCT_FWD_ANGLE_BLOCK  4 ... 4096 (powers of two)  angles per block of
 *                                 the forward's work order (128 with at least
 *                                 256 angles, else 8; at least the angles
 *                                 per workgroup)
 *   KCT_FWD_XCD_CHUNK    -1, 0, N  forward tiles an XCD takes per turn: -1
 *                                 one eighth of all in order, 0 half a row
 *                                 band of the angle block (with at least 256
 *                                 angles; else -1), N tiles
 *   KCT_FWD_PAD_F32      0 or 1   the forward widens a 16-bit volume into FP32
 *                                 padded copies (1 while those fit in 4 GiB)
 *   KCT_BWD_KZ           1, 8, 16 voxels per back-projector thread along z
 *   KCT_BWD_ACC          0 or 1   back-projector sums in registers or LDS (1)
 *   KCT_BWD_SPLIT        1..16    angle chunks of the back projection
 *                                 (more than 1 only for small volumes)
 *   KCT_BWD_RAYS         0 or 1   the ray-driven back projector (1 wherever
 *                                 every voxel's footprint is narrower than a
 *                                 pixel, which it needs; 1 is ignored
 *                                 elsewhere) or the voxel-driven one
 *   KCT_BWD_XCD_CHUNK    -1 or N  back-projector tiles an XCD takes per turn
 *                                 (-1: one contiguous eighth per XCD; by
 *                                 default whole rows of tiles, at least 32)
 *   KCT_BWD_TEST_PW_MAX  >= 1     test hook: caps the back projector's per-tile
 *                                 patch width, so that the footprint overflow
 *                                 report (kct_plan_check, history code 4) can
 *                                 be exercised; the sums are then truncated
 * The forward settings and KCT_BWD_XCD_CHUNK give bitwise-equal outputs;
 * they regroup only the per-workgroup partial sums that the solvers reduce.
 * KCT_BWD_SPLIT changes the order of the FP32 sums.
 */
kct_status kct_plan_create(const kct_geometry *geom, int device, kct_plan **out);

/* Free a plan and every device buffer it owns.  NULL is accepted. */
kct_status kct_plan_destroy(kct_plan *plan);

/*
 * Allocate the padded volume copies that plain kct_forward calls on volumes
 * stored in `vol_dtype` read: 2 (nx+2)(ny+2)(nz+2) elements (FP32 for
 * volumes the plan widens, else `vol_dtype`).  Nothing happens when the plan
 * already holds enough.  Synchronous: replacing smaller copies first waits for
 * the device.  Solves do not need this (they keep the copies in their
 * workspace).  KCT_E_OOM if the allocation fails.
 */
kct_status kct_plan_reserve(kct_plan *plan, int32_t vol_dtype);

/*
 * Synchronous check of the projector calls made on `plan` so far: waits for
 * `stream`, then reads and clears the plan's error flag.  KCT_OK, or
 * KCT_E_GEOMETRY when a back projection since the last check met a voxel
 * footprint wider than the plan's bounds (see Errors above) and returned
 * truncated sums.  Work on other streams must be finished by the caller.
 */
kct_status kct_plan_check(kct_plan *plan, void *stream);

/* Device bytes the plan holds now: its tables (per-angle geometry, 1/v per
 * detector row, the ray length of every detector pixel: nu * nv floats), the
 * back projector's partial volumes (small volumes) and the padded volume
 * copies of kct_plan_reserve. */
kct_status kct_plan_device_bytes(const kct_plan *plan, size_t *bytes);

/*
 * Forward projection (paper Sec. 2: every Krylov iteration applies A once):
 * d_proj = A d_vol.  d_vol: [nz][ny][nx] of `vol_dtype`; d_proj:
 * [n_angles][nv][nu] of `proj_dtype`, overwritten.  Ray sums accumulate in
 * FP32; ray geometry is evaluated in FP64.  Enqueued on `stream`.  The plan
 * must hold padded copies for `vol_dtype` (kct_plan_reserve); otherwise
 * KCT_E_BUDGET and nothing is enqueued.
 */
kct_status kct_forward(kct_plan *plan, const void *d_vol, int32_t vol_dtype, void *d_proj,
                       int32_t proj_dtype, void *stream);

/*
 * Forward projection that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and result as kct_forward
 * (bitwise: the same kernels), but the padded volume copies live in a device
 * array of KCT_NOALLOC_SCRATCH_BYTES that the library holds, on each GPU it
 * runs on, until the process ends; kct_plan_reserve is not needed.  The
 * copies take 2 (nx+2)(ny+2)(nz+2) elements of FP32 (for volumes the plan
 * widens, see KCT_FWD_PAD_F32) or of the volume's type: up to 254^3 voxels
 * in FP32.  Larger volumes: KCT_E_BUDGET, nothing enqueued.  KCT_E_DEVICE if
 * the array's device address could not be resolved when the plan was
 * created.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (each call rewrites all of it before reading it):
 * calls that overlap in time on one GPU, from any stream, thread or plan,
 * race, and their projections are undefined.  Enqueued on `stream`.
 */
#define KCT_NOALLOC_SCRATCH_BYTES (128u << 20)
kct_status kct_forward_noalloc(kct_plan *plan, const void *d_vol, int32_t vol_dtype, void *d_proj,
                               int32_t proj_dtype, void *stream);

/*
 * Back projection with the exact transpose of kct_forward (paper Sec. 2.1.4
 * and Sec. 4: a mismatched back projector degrades the Krylov methods):
 * d_vol = A^T d_proj.  Voxel-driven gather; FP32 accumulation.  Layouts as in
 * kct_forward; d_vol is overwritten.  For a small volume (too few voxel tiles
 * to fill the GPU) the angles are split over up to 16 chunks whose partial
 * volumes (allocated with the plan) are summed in chunk order.  Enqueued on
 * `stream`.
 */
kct_status kct_backproject(kct_plan *plan, const void *d_proj, int32_t proj_dtype, void *d_vol,
                           int32_t vol_dtype, void *stream);

/*
 * Unmatched back projection d_vol = B d_proj (paper Sec. 2.1.4: GPU
 * toolboxes back-project with an approximation B of A^T; AB- and BA-GMRES
 * take such a B as preconditioner).  Voxel-driven: the centre of each voxel
 * is projected onto the detector, the projection of every angle is
 * interpolated bilinearly there (zero outside the detector) and weighted by
 * V / (du dv) * (DSD / w)^2 * |d| / DSD, with w the voxel's depth along the
 * central ray and |d| the source-to-pixel distance at its image, so that B
 * equals A^T on smooth data.  Layouts and storage pairs as kct_backproject;
 * FP32 sums in angle order.  Enqueued on `stream`.
 */
kct_status kct_backproject_interp(kct_plan *plan, const void *d_proj, int32_t proj_dtype, void *d_vol,
                                  int32_t vol_dtype, void *stream);

/* ------------------------------------------------------------------------ */
/* Solvers                                                                   */
/* ------------------------------------------------------------------------ */

typedef enum kct_solver {
    KCT_CGLS = 0,        /* Sec. 2.1.1; damped by lambda (Sec. 2.2, augmented system) */
    KCT_LSQR = 1,        /* Sec. 2.1.2; damped by lambda                              */
    KCT_LSMR = 2,        /* Sec. 2.1.3; damped by lambda                              */
    KCT_HYBRID_LSQR = 3, /* Sec. 2.2.1; stores the basis V_k; lambda fixed or chosen
                            at every iteration (kct_lambda_rule)                    */
    KCT_IRN_TV_CGLS = 4, /* Sec. 2.3.1: IRN majorants of isotropic TV, inner CGLS     */
    KCT_AB_GMRES = 5,    /* Sec. 2.1.4: GMRES on A B (B = the chosen back projector
                            as right preconditioner); stores k+1 projection-space
                            basis vectors                                          */
    KCT_BA_GMRES = 6,    /* Sec. 2.1.4: GMRES on B A (left preconditioner); stores
                            k+1 volume-space basis vectors                         */
    KCT_SIRT = 7,        /* Sec. 3's algebraic baseline: x += lam V A^T W (b - A x),
                            W = 1 / (A 1), V = 1 / (A^T 1); lambda in (0, 2)       */
    KCT_OS_SART = 8,     /* SIRT's update over n_subsets ordered angle subsets per
                            iteration (subset s: angles a with a mod n_subsets = s) */
    KCT_HYBRID_FLSQR_TV = 9 /* Sec. 2.3.2, eq. (TV_standard_form): hybrid flexible
                            LSQR for the TV problem.  The IRN weights L_k of the
                            current iterate enter as the changing right
                            preconditioner E (L_k D)^+ (the A-weighted
                            pseudoinverse; E removes the A-weighted constant
                            part, x0 is the best constant), with (L_k D)^+
                            applied by tv_inner FP64 CG steps on D^T L_k^2 D
                            (four FP64 volumes of work space).  Stores
                            n_iter gradient-space vectors (3 volumes each), n_iter
                            volumes and n_iter+1 projections; lambda_k fixed or
                            chosen per iteration (kct_lambda_rule); FP32 only */
} kct_solver;

/* The back projector B of AB-/BA-GMRES.  Every other solver uses A^T. */
typedef enum kct_backprojector {
    KCT_BP_MATCHED = 0, /* the exact transpose A^T (kct_backproject)             */
    KCT_BP_INTERP = 1   /* the interpolating B of kct_backproject_interp          */
} kct_backprojector;

/* How hybrid LSQR and hybrid fLSQR-TV set the Tikhonov parameter lambda_k of
 * their projected problem (Sec. 2.2.2).  Every other solver takes
 * KCT_LAMBDA_FIXED.
 *   FIXED: lambda_k = params.lambda.
 *   GCV:   lambda_k minimises the GCV function of the projected problem
 *          (B_k, ||b|| e_1), searched on a log grid sigma_max * 10^[-7, 1]
 *          (81 points) and refined by 60 golden-section steps.
 *   DP:    lambda_k makes the projected residual equal noise_level * ||b||
 *          (discrepancy principle); 0 while even lambda = 0 leaves a larger
 *          residual, +inf (x = 0) when noise_level >= 1.
 * Both use the SVD of B_k (one-sided Jacobi in FP64 on the device); for
 * fLSQR-TV B_k is the upper Hessenberg matrix of the flexible process. */
typedef enum kct_lambda_rule {
    KCT_LAMBDA_FIXED = 0,
    KCT_LAMBDA_GCV = 1,
    KCT_LAMBDA_DP = 2
} kct_lambda_rule;

/* Columns of one history row (FP64), one row per iteration (for IRN-TV: per
 * inner iteration).
 *   [0] residual norm the method recurs: CGLS ||b - A x_k||, LSQR and hybrid
 *       ||[b;0] - [A; lam I] x_k||, fLSQR-TV the projected
 *       ||[bbar;0] - [A Z_k; lam I] y_k||, LSMR ||[A; lam I]^T r_k||,
 *       IRN-TV ||b - A x||,
 *       AB-GMRES ||b - A x_k||, BA-GMRES ||B (b - A x_k)||, SIRT ||b - A x_k||
 *       before update k+1, OS-SART sqrt(sum_s ||b_s - A_s x||^2) with each
 *       term taken just before subset s updates x;
 *   [1] alpha_k; [2] beta_k (the method's own two leading scalars; GMRES:
 *       H[k+1, k] and the k-th diagonal entry of the rotated Hessenberg matrix;
 *       fLSQR-TV: the norm of the new gradient-space vector before it is
 *       normalised and M[k+1, k]);
 *   [3] 1 if the method had broken down (zero norm) by this iteration, 2 if a
 *       scalar became non-finite, 3 if the explicit residual rule stopped it,
 *       4 if a back projection of the run met a footprint wider than the
 *       plan's bounds (its sums were truncated: x is not valid; see Errors at
 *       the top of this file), else 0;
 *   [4] lambda_k, the Tikhonov parameter of iteration k (the fixed lambda, or
 *       hybrid LSQR's GCV / DP choice; IRN-TV: the TV weight lambda). */
#define KCT_HIST_COLS 5

typedef struct kct_solve_params {
    int32_t solver;    /* kct_solver                                            */
    int32_t n_iter;    /* iterations (IRN-TV: ignored, tv_outer*tv_inner used)   */
    double lambda;     /* Tikhonov damping (CGLS/LSQR/LSMR/hybrid) or TV weight  */
    int32_t tv_outer;  /* IRN-TV outer iterations                               */
    int32_t tv_inner;  /* IRN-TV: inner CGLS iterations per outer iteration;
                          fLSQR-TV: CG steps per pseudoinverse application   */
    double tv_eps;     /* IRN-TV, fLSQR-TV: smoothing epsilon of the weights     */
    int32_t vec_dtype; /* storage of the vectors the projectors read and write:
                          KCT_F32, KCT_BF16 or KCT_F16; x is always FP32       */
    int32_t lambda_rule; /* kct_lambda_rule; not FIXED only for hybrid LSQR      */
    double noise_level;  /* DP: relative noise level ||e|| / ||b||, in (0, inf)  */
    int32_t backprojector; /* kct_backprojector; not MATCHED only for the GMRES  */
    int32_t n_subsets;   /* OS-SART: ordered subsets (1..n_angles); else 0      */
    uint32_t flags;      /* KCT_FLAG_* bits; unknown bits are KCT_E_INVALID_ARG  */
    int32_t reserved;    /* must be 0                                            */
} kct_solve_params;

/* Stop when the explicit residual ||b - A x_k|| grows (CGLS, LSQR, LSMR;
 * Sec. 3.1.1: the toolbox's guard against lost orthogonality and accumulated
 * rounding).  Costs one more forward projection per iteration.  When it
 * triggers, x is the iterate before the increase, history column 3 holds 3
 * from that row on, and column 0 holds the explicit residual throughout. */
#define KCT_FLAG_STOP_ON_RESIDUAL_INCREASE 1u

/* Record the explicit residual ||b - A x_k|| in history column 0 after every
 * iteration without stopping (CGLS, LSQR, LSMR; Sec. 3.1.1 compares it with
 * the recurred residual).  Costs one more forward projection per iteration.
 * Implied by KCT_FLAG_STOP_ON_RESIDUAL_INCREASE. */
#define KCT_FLAG_EXPLICIT_RESIDUAL 2u

/* Warm start: d_x holds x_0 on entry instead of being overwritten with 0
 * (CGLS, with or without damping; LSQR and LSMR with lambda = 0, which then
 * run on b - A x_0 and add their iterates to x_0; SIRT and OS-SART).  A
 * stationary method (SIRT, OS-SART) started from its own k-th iterate
 * continues its run exactly; a Krylov method starts a new Krylov space. */
#define KCT_FLAG_X0_GIVEN 4u

/* Workspace bytes kct_solve needs for `params` on `plan`. */
kct_status kct_solve_workspace_bytes(const kct_plan *plan, const kct_solve_params *params,
                                     size_t *bytes);

/*
 * Run a solver from x0 = 0 for a fixed number of iterations (the paper's
 * iterates live in K_k(A^T A, A^T b), Sec. 2).  d_b: FP32 projections
 * [n_angles][nv][nu]; d_x: FP32 volume [nz][ny][nx], overwritten with x_k.
 * d_ws: device workspace of at least kct_solve_workspace_bytes (contents
 * undefined on entry and exit).  d_history: device FP64 array of
 * n_rows * KCT_HIST_COLS, n_rows = n_iter (IRN-TV: tv_outer * tv_inner), or
 * NULL.  All Krylov scalars stay in device FP64 memory; nothing synchronises
 * the host inside the loop.  Enqueued on `stream`.
 */
kct_status kct_solve(kct_plan *plan, const kct_solve_params *params, const void *d_b, void *d_x,
                     void *d_ws, size_t ws_bytes, double *d_history, void *stream);

/* ------------------------------------------------------------------------ */
/* Iteration-level API (continuous-batching server, checkpoint tests)        */
/* ------------------------------------------------------------------------ */

typedef struct kct_state kct_state;

/*
 * Bind a solver run to caller buffers without running it: d_b, d_x, d_ws and
 * d_history as for kct_solve (they must stay valid until kct_state_destroy).
 * The state remembers `stream`; kct_state_step enqueues its work there.
 */
kct_status kct_state_create(kct_plan *plan, const kct_solve_params *params, const void *d_b, void *d_x,
                            void *d_ws, size_t ws_bytes, double *d_history, void *stream,
                            kct_state **out);

/* Enqueue up to `n_steps` more iterations (the first call also enqueues the
 * initialisation).  Returns at once; the host counts iterations enqueued, so
 * no device synchronisation is needed. */
/* (KCT_SOLVE_GRAPHS=1 in the environment at kct_state_create: a CGLS run
 * without flags captures its second iteration into a HIP graph and replays
 * it for the later steps.  That needs a stream that can be captured, not the
 * legacy default stream; otherwise, and on any capture failure, the kernels
 * are enqueued as usual.  The results are bitwise the same either way.) */
kct_status kct_state_step(kct_state *state, int32_t n_steps);

/* Iterations enqueued so far and whether all requested iterations are. */
kct_status kct_state_progress(const kct_state *state, int32_t *iters_enqueued, int32_t *finished);

/*
 * Checkpoint and resume (serving preemption, long runs).  A run's whole
 * device state lives in the caller's buffers: the workspace, x and the
 * history.  To checkpoint, make sure the initialisation and `iters_done`
 * iterations have been enqueued (kct_state_step, at least once), wait for
 * the stream, and copy every byte of the three buffers.  To resume, copy them
 * back into buffers of the same sizes (any addresses, any later time, a new
 * plan of the same geometry) and call kct_state_resume with the same params
 * and b: nothing is enqueued, and the following kct_state_step calls continue
 * with iteration iters_done + 1, bitwise as the uninterrupted run would.
 * 0 <= iters_done <= the run's iteration count; KCT_E_INVALID_ARG otherwise.
 * The other arguments are as for kct_state_create.
 */
kct_status kct_state_resume(kct_plan *plan, const kct_solve_params *params, const void *d_b, void *d_x,
                            void *d_ws, size_t ws_bytes, double *d_history, void *stream, int32_t iters_done,
                            kct_state **out);

/* Release a state (not the caller's buffers).  NULL is accepted. */
kct_status kct_state_destroy(kct_state *state);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* Static English name of a status. */
const char *kct_status_str(kct_status status);

/* Detail of the last failed call on this thread ("" if none); valid until
 * the next call on this thread. */
const char *kct_last_error(void);

/* Library version string. */
const char *kct_version(void);

/* ------------------------------------------------------------------------ */
/* Test hooks: launch shapes the plan logic chooses, read on the host        */
/* ------------------------------------------------------------------------ */

/* The back projector's shape for `geom` without touching a device: voxels per
 * thread along z, the unrolled column count, and the per-tile detector patch
 * bounds (columns, rows).  Any output may be NULL.  Returns a kct_status
 * (geometry validation as kct_plan_create). */
int kct_debug_bwd_shape_geom(const kct_geometry *geom, int *kz, int *ncmax, int *pw, int *ph);

/* The forward's shape for `geom` without touching a device: pixels per wave
 * row, angles per workgroup, angles per work-order block, and whether 16-bit
 * volumes are widened into FP32 padded copies (1) or not (0).  Returns a
 * kct_status. */
int kct_debug_fwd_shape_geom(const kct_geometry *geom, int *lane_u, int *wave_angles, int *angle_block,
                             int *pad_f32);

/* The back projector's shape of an existing plan (as kct_debug_bwd_shape_geom). */
void kct_debug_bwd_shape(const kct_plan *plan, int *kz, int *ncmax, int *pw, int *ph);

/* Which back projector the plan logic picks for `geom`, without touching a
 * device: the number of angle chunks (1, or up to 16 for small volumes) and
 * whether the ray-driven kernel runs (1: every voxel's footprint is narrower
 * than one pixel, so rays are walked through voxel tiles) or the
 * voxel-driven one (0).  Any output may be NULL.  Returns a kct_status. */
int kct_debug_bwd_mode_geom(const kct_geometry *geom, int *split, int *rays);

/* The same for an existing plan. */
void kct_debug_bwd_mode(const kct_plan *plan, int *split, int *rays);

#ifdef __cplusplus
}
#endif

#endif /* KCT_H */
