/*
 * caspar_ba.h -- C ABI of the MI355X (gfx950) bundle-adjustment hot path.
 *
 * The library solves the bundle-adjustment problem of the paper's Section VI-A
 * (Snavely reprojection factor: camera = pose + (f, k1, k2), point = R^3,
 * residual = predicted pixel - observed pixel) with the solver of Section V:
 * Levenberg-Marquardt with the gain-ratio damping update, tangent-space
 * linearisation and retraction, and the damped normal equations solved
 * directly (no Schur reduction) by block-Jacobi preconditioned conjugate
 * gradients on the normal equations (PCGNR), one preconditioner block per
 * camera and per point.
 *
 * Conventions shared by every call
 *  - Pointers marked (dev) are device pointers on the GPU that was current
 *    when the handle was created; (host) pointers are ordinary host memory.
 *    The caller owns every pointer it passes.  create() copies its inputs.
 *  - Cameras cross the boundary in BAL layout, 9 doubles per camera:
 *    angle-axis rotation (3), translation (3), f, k1, k2.  Points are 3
 *    doubles.  Observations are (camera index, point index, pixel x, y).
 *    Every array at the boundary is float64 and in the caller's order.
 *  - Tangent vectors (parity hooks, gradients) have length
 *    N = 9 n_cams + 3 n_points, laid out [cameras | points] in caller
 *    index order.  A camera's tangent is [dw(3), dt(3), df, dk1, dk2] with the
 *    rotation perturbed on the right, R <- R Exp(dw); everything else is
 *    additive.
 *  - Every call enqueues its GPU work on the HIP stream given at create()
 *    (NULL = the default stream) and returns when that work is complete.
 *  - Every call returns CASPAR_OK (0) or a negative status; the message of
 *    the last failure on the calling thread is caspar_last_error().  A failed
 *    call leaves the handle usable unless the status is CASPAR_EHIP.
 *  - Calls on one handle must not overlap (no internal locking).
 */
#ifndef CASPAR_BA_H
#define CASPAR_BA_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define CASPAR_API __attribute__((visibility("default")))
#else
#define CASPAR_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct caspar_ba caspar_ba; /* opaque handle */

/* Arithmetic of the hot path.
 * CASPAR_FP64: everything in float64.
 * CASPAR_FP32_MIXED: residuals, Jacobian blocks, the J / J^T products and the
 *   PCG vectors in float32; float64 for the cost sums, the gain ratio, the PCG
 *   dot products and alpha/beta, the block-Jacobi block sums and their
 *   inversion, and the parameters themselves. */
enum { CASPAR_FP64 = 0, CASPAR_FP32_MIXED = 1 };

/* Jacobian handling, OR-ed into the mode argument of create and
 * workspace_bytes.  By default the linearisation stores the 2x9 / 2x3 blocks
 * of every observation and each normal-equation product streams them from
 * HBM.  With CASPAR_RECOMPUTE_JACOBIAN nothing per observation is stored
 * beyond its indices: every product (and the adjoint) applies the blocks in
 * factored form from the camera row (rotation as a unit quaternion,
 * translation, calibration) and the point coordinates, without forming
 * them: 184 floating-point operations per observation instead of the 100
 * of applying stored blocks, against 96 (float32) or 192 (float64) bytes
 * of HBM traffic saved.  The map is the same linear operator; the results
 * agree with the stored-block ones to rounding (the rotation is rebuilt
 * from the quaternion), not bit for bit.  Sec. V notes that the generated
 * kernels exploit sparse and partially linear blocks; this is that idea
 * applied to the product. */
enum { CASPAR_RECOMPUTE_JACOBIAN = 0x10 };

/* Robust losses of the squared residual norm s = |r_o|^2 (caspar_ba_set_loss).
 * The paper's residual formulation leaves weighting schemes and robust losses
 * to the user (Sec. VI-A); these three, with scale c > 0 in pixels:
 *   CASPAR_LOSS_TRIVIAL  rho(s) = s
 *   CASPAR_LOSS_HUBER    rho(s) = s for s <= c^2, 2 c sqrt(s) - c^2 otherwise
 *   CASPAR_LOSS_CAUCHY   rho(s) = c^2 log(1 + s / c^2) */
enum { CASPAR_LOSS_TRIVIAL = 0, CASPAR_LOSS_HUBER = 1, CASPAR_LOSS_CAUCHY = 2 };

enum {
  CASPAR_OK = 0,
  CASPAR_EINVAL = -1,   /* bad argument, index out of range, non-finite input */
  CASPAR_EHIP = -2,     /* a HIP runtime call failed */
  CASPAR_ENOMEM = -3,   /* workspace smaller than caspar_ba_workspace_bytes() */
  CASPAR_ENUMERIC = -4, /* non-finite cost or PCG breakdown at the first step */
  CASPAR_EIO = -5       /* a file could not be opened, read or written */
};

/* Solver options; caspar_default_solve_opts() fills the defaults. */
typedef struct caspar_solve_opts {
  double lambda0;        /* initial damping; default 1e-2 = 1 / (trust radius 100, Sec. VI) */
  double pcg_tol;        /* PCG stops when ||b - A x||_2 <= pcg_tol ||b||_2; default 1e-3 (Sec. VI) */
  int32_t max_lm_iters;  /* LM iterations (an accepted or rejected trial each); default 20 */
  int32_t max_pcg_iters; /* PCG iteration cap per LM iteration; default 500 */
  double lambda_min;     /* damping clamp; default 1e-12 */
  double lambda_max;     /* default 1e16 */
  double grad_tol;       /* stop when ||g||_inf <= grad_tol * max(1, ||g_0||_inf); default 1e-12 */
  double min_cost;       /* stop when the cost F <= min_cost; default 1e-30 */
  int32_t pcg_check_every; /* host polls PCG convergence every this many iterations; within a
                              solve, the first poll of an LM step's PCG comes after
                              max(this, the previous step's PCG iterations - this); default 4 */
  int32_t flags;         /* reserved, 0 */
  double pred_tol;       /* stop when the step's predicted decrease pred <= pred_tol * F; default 0
                            (never).  Once pred falls below the resolution of F (about 1e-16 F) the
                            gain ratio is rounding noise; a few DBL_EPSILON stops the solve there
                            instead of accepting or rejecting steps by chance. */
} caspar_solve_opts;

/* Per-solve statistics (host). */
typedef struct caspar_solve_stats {
  int32_t lm_iters;        /* iterations run (accepted + rejected) */
  int32_t accepted;        /* accepted trials */
  int32_t pcg_iters_total; /* PCG iterations (matrix products) over all LM iterations */
  int32_t stop_reason;     /* 0 max iterations, 1 gradient, 2 cost, 3 predicted decrease */
  double initial_cost;     /* F = 1/2 sum |r|^2 at the start */
  double final_cost;       /* F at the returned parameters */
  double final_lambda;
  double seconds;          /* wall time of the solve (host clock, includes syncs) */
} caspar_solve_stats;

/* Per-LM-iteration record written by caspar_ba_solve when a history buffer
 * is given (host, max_lm_iters entries). */
typedef struct caspar_iter_record {
  double cost;        /* F after the iteration */
  double trial_cost;  /* F at theta (+) delta */
  double lambda;      /* damping used for this iteration's solve */
  double rho;         /* gain ratio (-inf when pred <= 0 or the trial is not finite) */
  double pred;        /* predicted decrease 1/2 (b^T d + d^T r_pcg + lambda d^T D d) */
  double pcg_rel_resid; /* ||r_pcg|| / ||b|| at exit */
  int32_t accepted;
  int32_t pcg_iters;
  double seconds;     /* host wall time from the start of the solve to the end of this
                         iteration (includes the relinearisation of an accepted step) */
} caspar_iter_record;

/* Fills opts with the defaults listed above (Sec. V solver, Sec. VI
 * settings: damping 1 / 100, CG tolerance 1e-3).  opts (host) must not be
 * NULL. */
CASPAR_API void caspar_default_solve_opts(caspar_solve_opts* opts);

/* Bytes of device workspace a handle of this size needs (0 on bad sizes).
 * Sec. V: the solver works in one block of GPU memory for the whole
 * optimisation, every array a view into it; here the caller allocates that
 * block and passes it to create().
 * n_obs must be < 2^31, n_cams < 2^25 and 3 n_points scalars (float64 or
 * float32 by precision) under 2 GiB.  mode = precision | Jacobian flag. */
CASPAR_API size_t caspar_ba_workspace_bytes(int32_t n_cams, int32_t n_points, int64_t n_obs, int mode);

/* Build a problem (paper Sec. VI-A: cameras, points, observations).
 * mode = CASPAR_FP64 or CASPAR_FP32_MIXED, optionally | CASPAR_RECOMPUTE_JACOBIAN.
 * cams (dev) [n_cams][9] BAL; points (dev) [n_points][3]; obs_cam, obs_pt
 * (dev) int32 [n_obs]; obs_px (dev) [n_obs][2].  workspace (dev, >= 256-byte
 * aligned, caspar_ba_workspace_bytes() long) must outlive the handle; the
 * library never allocates device memory of its own (the handle keeps one
 * small pinned host buffer for reading back solver scalars, freed by
 * caspar_ba_destroy).  Inputs are validated
 * (indices in range, values finite -> CASPAR_EINVAL).  The observations are
 * reordered internally (point-major, points grouped by their least-observed
 * camera); that order never shows at the boundary. */
CASPAR_API int caspar_ba_create(caspar_ba** out, int32_t n_cams, int32_t n_points, int64_t n_obs,
                     const double* cams, const double* points, const int32_t* obs_cam,
                     const int32_t* obs_pt, const double* obs_px, int mode,
                     void* workspace, size_t workspace_bytes, void* hip_stream);

/* create() without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The handle's workspace is a static
 * device array of the library, 256 MiB (268435456 bytes), which every GPU the
 * library runs on holds until the process ends; the call makes no device or
 * pinned-host allocation (scalar read-backs go through the handle's own host
 * memory, so solves poll a little slower than with create()).  Problems
 * whose caspar_ba_workspace_bytes() exceeds 256 MiB get CASPAR_ENOMEM (about
 * 1.4 million observations in CASPAR_FP32_MIXED | CASPAR_RECOMPUTE_JACOBIAN
 * mode at 6.5 observations per point; about 1.2 million with stored blocks
 * or float64 and recomputed blocks, 0.8 million in float64 with stored
 * blocks).  The array belongs to one
 * handle at a time on each GPU: while a handle created this way lives, a
 * second call on the same GPU returns CASPAR_EINVAL (destroy the first);
 * caspar_ba_destroy releases it.  The contents left by the previous handle
 * are overwritten by create, as with a fresh workspace.  Every other argument
 * and every later call on the handle behave as with caspar_ba_create on the
 * current device. */
CASPAR_API int caspar_ba_create_static(caspar_ba** out, int32_t n_cams, int32_t n_points, int64_t n_obs,
                                       const double* cams, const double* points, const int32_t* obs_cam,
                                       const int32_t* obs_pt, const double* obs_px, int mode, void* hip_stream);

/* Run Levenberg-Marquardt from the current parameters (Sec. V).  opts may be
 * NULL (defaults).  stats (host) may be NULL; history (host) may be NULL or
 * hold opts->max_lm_iters records.  The parameters afterwards are the last
 * accepted ones.  Returns CASPAR_ENUMERIC if the initial cost is not finite. */
CASPAR_API int caspar_ba_solve(caspar_ba* h, const caspar_solve_opts* opts, caspar_solve_stats* stats,
                    caspar_iter_record* history);

/* Current parameters (the nodes of the Sec. VI-A problem: camera poses with
 * their calibration, and points) in BAL layout, caller order (dev outputs;
 * either may be NULL). */
CASPAR_API int caspar_ba_get_params(caspar_ba* h, double* cams, double* points);

/* Replace the parameters (the nodes of the Sec. VI-A problem; dev inputs,
 * BAL, caller order; either may be NULL to keep that part).  Use with
 * lambda0 = the last final_lambda for a warm restart of the Sec. V solver. */
CASPAR_API int caspar_ba_set_params(caspar_ba* h, const double* cams, const double* points);

/* Select the robust loss (default CASPAR_LOSS_TRIVIAL).  The cost becomes
 * F = 1/2 sum_o rho(|r_o|^2) and every linearisation is iteratively
 * reweighted: with w_o = rho'(|r_o|^2) held fixed until the next
 * linearisation, residuals and Jacobian blocks are scaled by sqrt(w_o), so the
 * normal equations are (J^T W J + lambda D) delta = -J^T W r with
 * D = clamp(diag J^T W J) and J^T W r the exact gradient of F.  The gain
 * ratio compares the decrease of F with that weighted model's prediction.
 * The parity hooks (linearize, matvec, pcg, cost_fp64) and the adjoint use
 * the same weighted system; the adjoint holds the weights fixed.  scale must
 * be finite and > 0 (CASPAR_EINVAL otherwise, or for an unknown kind). */
CASPAR_API int caspar_ba_set_loss(caspar_ba* h, int32_t kind, double scale);

/* Replace the observed pixels, the measurements of the Sec. VI-A
 * reprojection factors (dev [n_obs][2], caller order); the structure (which
 * camera sees which point) is kept.  CASPAR_EINVAL for a non-finite value. */
CASPAR_API int caspar_ba_set_observations(caspar_ba* h, const double* obs_px);

/* Implicit adjoint of the optimum with respect to the observed pixels: the
 * implicit function theorem applied to the fixed point that the solver of
 * Sec. V converges to, J^T r = 0 at the optimum, with the Gauss-Newton
 * matrix of that solver (second-order residual terms dropped) and its
 * damping.  With g the tangent gradient of a loss L(cameras*, points*),
 * solve (J^T J + lambda_adj D) v = g by the same block-Jacobi PCG and write
 * dL/dpx_o = J_o v (dev [n_obs][2], caller order), since dr/dpx = -I.
 * grad_cams (dev [n_cams][9], BAL: gradient w.r.t. the angle-axis vector,
 * translation, f, k1, k2; may be NULL = 0) is mapped to the right tangent
 * with the inverse right Jacobian of SO(3); grad_points (dev [n_points][3],
 * may be NULL = 0).  J and D are those of the current parameters.  In
 * CASPAR_FP32_MIXED mode v and the PCG vectors are float32 (dots float64),
 * as in the forward solve.
 * flags: CASPAR_ADJ_GAUGE_PROJECT removes the D-weighted component of g
 * along the 7 similarity-gauge directions N (world rotation, translation,
 * scale): g <- g - D N (N^T D N)^-1 N^T g.  Because J N = 0 and
 * A N = lambda_adj D N this leaves J A^-1 g unchanged, and it keeps v free
 * of the 1/lambda_adj gauge component, so small lambda_adj stay well
 * conditioned.  pcg_iters and rel_resid (host, each may be NULL) receive the
 * iteration count and ||g - A v|| / ||g|| of the PCG recurrence at exit:
 * a rel_resid above pcg_tol means the solve stopped at max_pcg_iters and the
 * gradient is correspondingly inexact (the call still succeeds). */
enum { CASPAR_ADJ_GAUGE_PROJECT = 1 };
CASPAR_API int caspar_ba_backward(caspar_ba* h, const double* grad_cams, const double* grad_points,
                       double lambda_adj, double pcg_tol, int32_t max_pcg_iters, int32_t flags,
                       double* grad_obs_px, int32_t* pcg_iters, double* rel_resid);

/* ---- Parity hooks: single steps of the hot path at the current parameters ---- */

/* Linearise as the Sec. V solver does at each accepted step: the
 * tangent-space Jacobian blocks of the Sec. VI-A factor (residuals, Jacobian blocks, cost, gradient g = J^T r, damping
 * diagonal D = clamp(diag J^T J, 1e-6, 1e32)); with a robust loss the
 * residuals and blocks are the sqrt(w)-scaled ones and the cost is
 * 1/2 sum rho(|r|^2) (see caspar_ba_set_loss).  cost (host) may be NULL;
 * resid (dev [n_obs][2]), jac_cam (dev [n_obs][2][9]), jac_pt
 * (dev [n_obs][2][3]), grad (dev [N]) and diag (dev [N]) may each be NULL.
 * Outputs are float64 in caller order (FP32_MIXED values are widened). */
CASPAR_API int caspar_ba_linearize(caspar_ba* h, double* cost, double* resid, double* jac_cam,
                        double* jac_pt, double* grad, double* diag);

/* The damped normal-equation product the Sec. V solver's PCG applies without
 * forming J^T J or a Schur complement:
 * w = (J^T J + lambda D) p with J, D of the last linearisation (linearises
 * first if the parameters changed).  p, w (dev [N]); pAp (host, may be NULL)
 * receives p^T w as accumulated by the fused kernel. */
CASPAR_API int caspar_ba_matvec(caspar_ba* h, double lambda, const double* p, double* w, double* pAp);

/* The block-Jacobi preconditioner of Sec. V, one block per node (a 9x9 block
 * per camera, a 3x3 block per point): z = M^-1 r with M the block diagonal
 * of J^T J + lambda D (dev [N]). */
CASPAR_API int caspar_ba_block_jacobi_apply(caspar_ba* h, double lambda, const double* r, double* z);

/* The inner solve of Sec. V, block-Jacobi preconditioned conjugate gradients
 * on the normal equations:
 * PCG on (J^T J + lambda D) x = b from x = 0 (dev [N]); iters and rel_resid
 * (host, may be NULL) receive the iteration count and ||r||/||b|| of the
 * recurrence residual. */
CASPAR_API int caspar_ba_pcg(caspar_ba* h, double lambda, const double* b, double tol, int32_t max_iters,
                  double* x, int32_t* iters, double* rel_resid);

/* The objective the Sec. V solver minimises over the Sec. VI-A factors:
 * cost F = 1/2 sum |r|^2 at the current parameters, accumulated in float64
 * from residuals evaluated in float64 regardless of the handle's precision
 * (host out). */
CASPAR_API int caspar_ba_cost_fp64(caspar_ba* h, double* cost);

/* Predicted pixels of the Snavely model (Sec. VI-A) for arbitrary parameters, float64,
 * no handle needed (dev in/out, caller layout).  hip_stream may be NULL. */
CASPAR_API int caspar_project(int32_t n_cams, int32_t n_points, int64_t n_obs, const double* cams,
                   const double* points, const int32_t* obs_cam, const int32_t* obs_pt,
                   double* px_out, void* hip_stream);

/* Sizes of the internal layout (host outs, any may be NULL; a helper for
 * measurement, no passage of the paper defines it): the number of
 * cameras accumulated in LDS by the fused product, observations of the other
 * cameras, wave tiles, and workgroups of the fused product. */
CASPAR_API int caspar_ba_layout_info(caspar_ba* h, int32_t* hot_cams, int64_t* cold_obs, int64_t* n_tiles,
                          int32_t* matvec_groups);

/* Kernel timing for roofline reporting (Sec. VI compares solvers by time;
 * this times the product that dominates it).  While enabled, every k-th launch of
 * the fused normal-equation product made by solve/pcg/backward/matvec
 * (counted across solves, so every position inside a solve is sampled) is
 * timed by HIP events on the handle's stream that the launch itself stamps;
 * launches that found the PCG already finished (no work) are not counted. */
typedef struct caspar_timing {
  int64_t matvec_launches;  /* timed fused-product launches that did work */
  double matvec_ms;         /* summed duration of those launches (event time) */
  double matvec_bytes;      /* bytes one launch must move: per observation the
                               24 Jacobian scalars (stored mode) and two int32
                               indices; per parameter p and D read, w written;
                               recompute mode adds the camera rows and the
                               float64 points instead of the blocks */
} caspar_timing;

/* enable = k > 0 starts (and zeroes) the counters and times every k-th
 * launch of the fused product from here on (k = 1: every launch; the events
 * themselves leave the GPU idle for a few microseconds per launch, so a
 * larger k disturbs a timed solve less); 0 stops them; k < 0 is
 * CASPAR_EINVAL.  matvec_launches then counts the timed launches. */
CASPAR_API int caspar_ba_set_timing(caspar_ba* h, int enable);
CASPAR_API int caspar_ba_get_timing(caspar_ba* h, caspar_timing* out);

/* Release the handle (its pinned host read-back buffer and HIP events; the
 * caller's workspace is untouched and may be freed afterwards).  NULL is a
 * no-op. */
CASPAR_API void caspar_ba_destroy(caspar_ba* h);

/* Pose between-factors: a second factor type on pairs of cameras (the
 * paper's solvers take any collection of factor types, an odometry factor
 * being its example, Section V).  Factor f between cameras a = cam_i[f] and
 * b = cam_j[f] (caller indices, a != b) with measured relative pose
 * Z = meas[f] = (angle-axis (3), translation (3)) of T_b T_a^-1 (world-to-
 * camera poses T = (R, t)) and square-root weights weights[f] = (s_rot,
 * s_trans) > 0 has the residual
 *   r = [ s_rot   Log(Z_R^T R_b R_a^T) ;  s_trans (t_b - R_b R_a^T t_a - Z_t) ]
 * and adds 1/2 |r|^2 to the cost.  The factors enter the linearisation
 * (gradient, camera blocks, damping diagonal), every product, the trial
 * cost, caspar_ba_cost_fp64, solve and backward; robust losses apply to the
 * reprojection factors only.  The parity hook caspar_ba_linearize still
 * exports the reprojection residuals and blocks alone (its g and D include
 * the factors).  backward() refuses CASPAR_ADJ_GAUGE_PROJECT while factors
 * are set: they fix the scale, so the similarity gauge is no longer free.
 *
 * between_workspace_bytes: device bytes set_between needs for n_factors on a
 *   problem of n_cams cameras.
 * set_between: copies the factors (host arrays: cam_i, cam_j [n], meas
 *   [n][6], weights [n][2]) into dev_workspace (dev, 256-byte aligned, at
 *   least between_workspace_bytes; the caller owns it and keeps it alive
 *   until the handle is destroyed or set_between is called again).  Replaces
 *   any earlier set; n_factors = 0 removes them (the workspace may then be
 *   NULL).  The next solve/linearize re-linearises.  CASPAR_EINVAL for an
 *   index out of range, equal cameras, a non-finite measurement, a weight
 *   that is not finite and positive, or a workspace that is too small or
 *   misaligned. */
CASPAR_API size_t caspar_ba_between_workspace_bytes(int32_t n_factors, int32_t n_cams);
CASPAR_API int caspar_ba_set_between(caspar_ba* h, int32_t n_factors, const int32_t* cam_i,
                                     const int32_t* cam_j, const double* meas, const double* weights,
                                     void* dev_workspace, size_t workspace_bytes);

/* BAL problem files.  The paper evaluates on the Bundle Adjustment in the
 * Large datasets (Section VI); these calls read and write their text format,
 * a stream of whitespace-separated tokens:
 *   n_cams n_points n_obs
 *   n_obs records    camera_index point_index x y
 *   n_cams records   9 values: angle-axis rotation (3), translation (3), f, k1, k2
 *   n_points records 3 values
 * which is the boundary's own layout, so the arrays go to create() as they
 * are.  All pointers are (host) and owned by the caller; no GPU is touched.
 *
 * read_header: the three counts of the file at path (outs may be NULL).
 * read: the whole problem into caller arrays sized from the header:
 *   obs_cam[n_obs], obs_pt[n_obs] (int32), px[n_obs][2], cams[n_cams][9],
 *   points[n_points][3] (float64).  The sizes passed must equal the header's.
 *   Reals are parsed correctly rounded, so a file written with round-trip
 *   precision reads back bit for bit.  The file is tokenised by up to 16 host
 *   threads.
 * write: the same arrays to path (created or truncated), every real in its
 *   shortest round-trip form.
 * Errors: CASPAR_EIO when the file cannot be opened, read or written;
 * CASPAR_EINVAL for a malformed header, a token that is not a number, a
 * non-finite value, an index out of range, too few or too many values, sizes
 * that differ from the header, or a NULL array; the message names the
 * offending record.  A failed read may leave the output arrays partly
 * written. */
CASPAR_API int caspar_bal_read_header(const char* path, int32_t* n_cams, int32_t* n_points, int64_t* n_obs);
CASPAR_API int caspar_bal_read(const char* path, int32_t n_cams, int32_t n_points, int64_t n_obs,
                               int32_t* obs_cam, int32_t* obs_pt, double* px, double* cams, double* points);
CASPAR_API int caspar_bal_write(const char* path, int32_t n_cams, int32_t n_points, int64_t n_obs,
                                const int32_t* obs_cam, const int32_t* obs_pt, const double* px,
                                const double* cams, const double* points);

/* Message of the last failed call on this thread ("" if none). */
CASPAR_API const char* caspar_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CASPAR_BA_H */
