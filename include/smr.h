/*
 * smr.h -- C ABI of the MI355X (gfx950) library for sine-transform-preconditioned
 * MINRES on the time-flipped all-at-once systems of the heat equation
 * (S. Hon, P. Y. Fung, J. Dong, S. Serra-Capizzano, arXiv 2201.10062).
 *
 * Problem (Sec. 1, eqn:heat): u_t = div(a grad u) + f on (0,1)^dim x (0,T], u = 0 on
 * the boundary, u(.,0) = u0, discretised by finite differences on N interior points
 * per axis (h = 1/(N+1), m = N^dim unknowns per time level, M = I) and n time steps
 * (tau = T/n) with
 *   - the theta-method (eq. theta): T_H has A0 = I + theta tau K on the block
 *     diagonal and A1 = -I + (1-theta) tau K below it;
 *   - BDF-l, l = 2, 3, 4 (eqn:matrix_gen): A0 = alpha_0 I + tau K, A_k = alpha_k I.
 * K = K(a) is the 3-point (1D), 5-point (2D) or 7-point (3D, the setting of Sec. 5's
 * Example 3) stencil of eqn:matrix_Km_va built from face values of a.  The library solves Y T u = Y f_H (eqn:main_system, Y the time
 * flip) by preconditioned MINRES with
 *   - SMR_P_H: P_H (def:matrix_P) or, for BDF-l, Phat (def:matrix_P_gen); for
 *     variable a the averaged Toeplitz Kbar of Sec. 3.1.1 replaces K inside P only.
 *     P^{-1} = (S_n (x) U) diag(1/sigma) (S_n (x) U), U the spatial sine transform,
 *     sigma_{j,k} = |ghat(phi_j)| evaluated at the eigenvalue mu_k of K (or Kbar);
 *   - SMR_P_THETA_CHEB: P_theta (def:matrix_mod_P) whose per-time-mode SPD solves
 *     (eta_j I + tau zeta_j K(a)) are replaced by k steps of Chebyshev iteration
 *     preconditioned by eta_j I + tau zeta_j abar K_lap (the paper leaves the inner
 *     solver open).  For constant a that inner preconditioner is exact, and P_theta^{-1}
 *     is the sine-basis division by eta_j + tau zeta_j mu_k (one step solves each mode);
 *   - SMR_P_NONE: identity.
 *
 * Conventions shared by every entry point
 *   Layout: every vector is float64, C-ordered (time, [z,] y, x), x fastest; a solution /
 *     right-hand side has n*m entries, a source f has (n+1)*m (levels t_0..t_n).
 *   Pointers: arguments named d_* or documented "device" are device pointers on the
 *     current HIP device; "host" pointers are ordinary host memory.  The caller owns
 *     every buffer.  The library never allocates device memory: all scratch lives in
 *     the caller's workspace (size from smr_workspace_size).
 *   Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it.  smr_setup and the solves synchronise it before
 *     returning; the apply/build/grad calls are asynchronous.
 *   Concurrency: one call in flight per plan (a plan owns its workspace, its captured
 *     iterations and its pinned status buffer).  Calls on distinct plans with distinct
 *     workspaces are independent and may run from different threads.  The batched solves
 *     share one capture stream, graph cache and pinned status buffer per device; the
 *     library serialises them (a batched call waits for any other batched call on the same
 *     device to return).  smr_profile_enable / smr_profile_read are process-wide and not
 *     thread-safe (diagnostics only).
 *   Errors: every call returns an smr_status; no exception crosses the ABI.  On any
 *     status other than SMR_OK a human-readable reason is available from
 *     smr_last_error() (thread-local, valid until the next call on the thread).
 *   Limits: dim in {1, 2, 3}; N + 1 a power of two with 2 <= N + 1 <= 512 (<= 128 in 3D);
 *     1 <= n <= 1024 (n >= l for BDF-l); 0 <= theta <= 1; every face value finite and > 0.
 */
#ifndef SMR_H
#define SMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smr_plan smr_plan;

typedef enum {
  SMR_OK = 0,
  SMR_EINVAL = 1,        /* bad descriptor, pointer or argument                         */
  SMR_EWORKSPACE = 2,    /* workspace missing, too small or not 256-byte aligned        */
  SMR_EDEVICE = 3,       /* a HIP runtime error (message in smr_last_error)             */
  SMR_ENOTSPD = 4,       /* gamma^2 <= 0 or not finite: P is not SPD on the residual    */
  SMR_EBREAKDOWN = 5,    /* Lanczos/QR breakdown with a non-zero residual               */
  SMR_ENOTCONV = 6,      /* maxit reached; x holds the last iterate, info is filled     */
  SMR_EUNSUPPORTED = 7   /* valid request that the library does not implement         */
} smr_status;

/* Time discretisation: the theta method, or the l-step backward difference formula BDF-l
 * (Sec. 4, eqn:matrix_gen; the enum value is l), A_(0) = alpha_0 I + tau K, A_(k) = alpha_k I
 * with alpha_k the coefficients of sum_{j=1}^{l} nabla^j / j (BDF2: 3/2, -2, 1/2; BDF3: 11/6,
 * -3, 3/2, -1/3; BDF4: 25/12, -4, 3, -4/3, 1/4).  BDF right-hand sides are given directly
 * (start-up values belong in them). */
typedef enum { SMR_THETA = 0, SMR_BDF2 = 2, SMR_BDF3 = 3, SMR_BDF4 = 4 } smr_scheme;
typedef enum { SMR_P_H = 0, SMR_P_THETA_CHEB = 2, SMR_P_NONE = 3 } smr_precond;
/* Arithmetic inside P^{-1} during the solves.  The matvec, the Lanczos recurrences, the
 * MINRES scalars and the true residual are always float64.  SMR_FP32 runs the time-axis sine
 * transforms of P^{-1} on the float32 matrix cores with float32 accumulation: in the sine
 * basis (see SMR_FLAG_GENERAL_PATH) z is also stored in float32; on the physical-basis path
 * (P_H, Phat, P_theta) every intermediate vector of P^{-1} (after each spatial transform pass
 * and each per-mode Chebyshev step) is stored in float32, while the spatial transforms, the
 * 1/sigma scaling and the Chebyshev updates compute in float64.  SMR_EINVAL with SMR_P_NONE.
 * smr_apply_P_inv always applies P^{-1} in float64. */
typedef enum { SMR_FP64 = 0, SMR_FP32 = 1, SMR_BF16 = 2 } smr_pprec;
/* P_H / Phat solves run in the spatial sine basis (b and x0 transformed on entry, x on exit;
 * the same iterates in exact arithmetic): for constant a, Y T and P^{-1} act per spatial mode
 * and one fused kernel does a MINRES iteration (so do P_theta solves of a constant a, whose
 * per-mode blocks are then diagonal in that basis); for a variable a in 2D with N + 1 in
 * {32, 64, 128} (Kbar inside P, Sec. 3.1.1), a per-time-level kernel first applies
 * U K(a) U (sine transforms held in LDS) and the fused kernel takes that matvec.  Other
 * variable-coefficient cases, P_theta of a variable a and P = I run the general
 * physical-basis iteration (stencil matvec and space-time transforms), which this flag
 * forces for every plan. */
#define SMR_FLAG_GENERAL_PATH 1
/* Column-tile width of the fused sine-basis kernel: each workgroup owns that many spatial
 * modes of all n time levels (the folded time blocks of Sec. 3.1.1 are contracted per tile
 * on the matrix cores).  With neither bit set, smr_setup times one steady iteration at each
 * width on the plan's own workspace and keeps 32 unless 16 is at least 5% faster (narrow
 * tiles pay off when the spatial grid is small; with ceil(n/2) <= 64 a 64-mode tile is a
 * third candidate, for large grids with few time levels); the choice is cached per device
 * and shape (see smr_tune_stats); batched calls time each class of instances the same way.
 * 32 needs ceil(n/2) <= 128 and 64 (SMR_FLAG_TILE64) ceil(n/2) <= 64, or <= 128 with SMR_FP32
 * (SMR_EUNSUPPORTED otherwise);
 * ceil(n/2) > 128 always takes 16.  The width changes only the summation order of the
 * reductions.  Setting more than one of the three bits is SMR_EINVAL. */
#define SMR_FLAG_TILE16 2
#define SMR_FLAG_TILE32 4
#define SMR_FLAG_TILE64 128
/* Variant of the physical-basis P^{-1} (no effect on the sine-basis path): 8-line (PINV_F64)
 * or 16-line (PINV_F64_COL16) tiles in the spatial transform's column passes with float64
 * intermediate vectors, and for SMR_FP32 plans float32 intermediate vectors with 8-line
 * (PINV_F32) or 16-line (PINV_F32_COL16) column tiles (float64 intermediates of an SMR_FP32
 * plan keep float32 GEMMs in the time transform).  16-line tiles apply to 2D plans with
 * N + 1 in {32, ..., 256} (others take the 8-line form).  With none set, smr_setup times a
 * few P^{-1} applications of each candidate on the plan's workspace and keeps the fastest
 * (PINV_F64 unless another is 3% faster), cached per device and shape; smr_pinv_variant
 * reports the choice.  At most one; the float32 ones need SMR_FP32 (else SMR_EINVAL). */
#define SMR_FLAG_PINV_F64 8
#define SMR_FLAG_PINV_F32 16
#define SMR_FLAG_PINV_F32_COL16 32
#define SMR_FLAG_PINV_F64_COL16 64
/* Form of the per-level matvec U K(a) U of an N = 127 variable-coefficient 2D solve in the
 * sine basis (Sec. 3.1.1: the spatial sine transform diagonalises the constant part; for a
 * variable a each time level goes through U, the 5-point K(a) of eqn:matrix_Km_va, and U):
 * MATVEC_LEVEL holds a whole level in LDS per workgroup (one workgroup per CU);
 * MATVEC_TILES streams three passes over 16-line tiles (rows of the source, columns with the
 * stencil, rows into (T z)^), with four level-sized intermediates in the workspace, so that
 * several workgroups share a CU.  With neither set, smr_setup times both on the plan's
 * workspace and keeps the tiled passes unless the level form is 3% faster, cached per device
 * and shape; smr_matvec_tiles reports the choice.  Same arithmetic; only the grouping of the
 * partial sums differs.  No effect on other plans.  At most one (else SMR_EINVAL). */
#define SMR_FLAG_MATVEC_LEVEL 256
#define SMR_FLAG_MATVEC_TILES 512

typedef struct {
  int32_t dim;             /* spatial dimension, 1, 2 or 3                                */
  int32_t N;               /* interior points per axis                                    */
  int32_t n;               /* time steps                                                  */
  int32_t scheme;          /* smr_scheme                                                  */
  int32_t precond;         /* smr_precond                                                 */
  int32_t pprec;           /* smr_pprec                                                   */
  int32_t cheb_k;          /* Chebyshev steps per mode (SMR_P_THETA_CHEB), 1..16          */
  int32_t flags;           /* SMR_FLAG_* bits: GENERAL_PATH (iterate in the physical basis
                            * even when a is constant), TILE16/32/64 (fix the column-tile
                            * width), PINV_* (the physical-basis P^{-1} variant),
                            * MATVEC_LEVEL/TILES (the N = 127 per-level matvec form);
                            * other bits must be 0 (SMR_EINVAL)                          */
  double T;                /* final time (> 0)                                            */
  double theta;            /* theta-method parameter (SMR_THETA)                          */
  /* Coefficient a (host pointers, copied during smr_setup).  Give at most one form:
   *   face values: dim 1: ax[N+1], ax[i] = a((i+1/2)h);
   *                dim 2: ax[N][N+1], ax[j][i] = a((i+1/2)h, (j+1)h) and
   *                       ay[N+1][N], ay[j][i] = a((i+1)h, (j+1/2)h);
   *                dim 3: ax[N][N][N+1], ax[k][j][i] = a((i+1/2)h, (j+1)h, (k+1)h),
   *                       ay[N][N+1][N], ay[k][j][i] = a((i+1)h, (j+1/2)h, (k+1)h) and
   *                       az[N+1][N][N], az[k][j][i] = a((i+1)h, (j+1)h, (k+1/2)h);
   *   nodal values (dim 1, 2): a_nodal[(N+2)^dim] on the grid including the boundary; each
   *                 face takes the mean of its two end nodes;
   *   all NULL: a = 1. */
  const double *ax_host;
  const double *ay_host;
  const double *a_nodal_host;
  const double *az_host;   /* dim 3 face values along z (with ax_host, ay_host); else NULL */
} smr_desc;

typedef struct {
  int32_t iters;           /* MINRES iterations performed (= matrix-vector products)     */
  int32_t status;          /* smr_status of the solve                                     */
  double relres_true;      /* ||f_H - T x||_2 / ||f_H||_2 at exit (float64 matvec)        */
  double relres_prec;      /* |eta| / gamma_1: relative P^{-1}-norm residual estimate     */
  int32_t res_evals;       /* true residuals evaluated (the initial one included); the
                              sine-basis path skips those that sqrt(min sigma) |eta| proves
                              to exceed the tolerance                                     */
  int32_t tile_cols;       /* column-tile width of the fused sine-basis launches the solve ran
                              with (a batch class's timed width; 0 on the physical-basis path) */
} smr_info;

/* Bytes of device workspace needed by a plan for `desc` (Sec. 3.1.1: O(nm) storage). */
smr_status smr_workspace_size(const smr_desc *desc, size_t *bytes);

/* Validate `desc`, build the plan's tables (face values, Kbar averages, sine-transform
 * eigenvalues, the folded time sine matrix, FFT twiddles) on the host and copy them into
 * the caller's device workspace `d_ws` (>= smr_workspace_size bytes, 256-byte aligned,
 * owned by the caller and kept alive until smr_destroy).  Synchronises `stream`. */
smr_status smr_setup(const smr_desc *desc, void *d_ws, size_t ws_bytes, void *stream,
                     smr_plan **out);

/* Column-tile width the plan's sine-basis solves launch with (16, 32 or 64; see
 * SMR_FLAG_TILE16), 0 when its solves run in the physical basis.  Host only. */
smr_status smr_tile_cols(const smr_plan *plan, int32_t *cols);

/* The physical-basis P^{-1} variant of a plan (see SMR_FLAG_PINV_F64): 0 float64
 * intermediates, 1 float32, 2 float32 with 16-line column tiles, 3 float64 with 16-line
 * column tiles; -1 for plans whose solves run in the sine basis or without a preconditioner.
 * Host only. */
smr_status smr_pinv_variant(const smr_plan *plan, int32_t *variant);

/* 1 when the plan's per-level matvec runs as tiled passes (see SMR_FLAG_MATVEC_TILES), else 0
 * (level form, or a plan without that matvec).  Host only. */
smr_status smr_matvec_tiles(const smr_plan *plan, int32_t *tiled);

/* The autotuner's cache (host, process-wide): shapes timed so far (entries), and how many
 * set-ups and batched calls found their choice cached (hits) or timed it (misses).
 * smr_tune_reset clears it (the next plans and batches time their choices again). */
smr_status smr_tune_stats(int64_t *entries, int64_t *hits, int64_t *misses);
smr_status smr_tune_reset(void);

/* Free the host-side plan (the workspace stays with the caller).  NULL is accepted. */
smr_status smr_destroy(smr_plan *plan);

/* f_H of Sec. 1 (theta scheme): b_k = theta tau f^(k) + (1-theta) tau f^(k-1), k = 1..n,
 * plus (I - (1-theta) tau K) u0 on block 1.  d_f: (n+1)*m, d_u0: m (NULL = 0),
 * d_b: n*m (output, unpermuted).  SMR_EINVAL for the BDF schemes (their b is given). */
smr_status smr_build_rhs(const smr_plan *plan, const double *d_f, const double *d_u0,
                         double *d_b, void *stream);

/* d_y = Y T d_x (eqn:main_system, eqn:main_system_gem_sym); d_x, d_y: n*m, distinct. */
smr_status smr_apply_A(const smr_plan *plan, const double *d_x, double *d_y, void *stream);

/* d_z = P^{-1} d_v for the plan's preconditioner and pprec; d_v, d_z: n*m.  In-place
 * (d_z == d_v) is allowed. */
smr_status smr_apply_P_inv(const smr_plan *plan, const double *d_v, double *d_z, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): d_z = P^{-1} d_v exactly as
 * smr_apply_P_inv (same kernels, same result bit for bit), but its intermediate vectors live
 * in a static device array owned by the library, SMR_STATIC_SCRATCH_BYTES per GPU, held until
 * the process ends, instead of the plan's workspace.  The call allocates nothing.  It needs
 * 2 (P_H, Phat) or 4 (P_theta) vectors of n*m doubles, each rounded up to 256 bytes, within
 * that size (SMR_EINVAL beyond it; n*m <= 4194304 for P_H, 2097152 for P_theta); P = I needs
 * none.  Every call on a GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, threads or processes' streams on this library instance) race and
 * corrupt each other's results; serialise them, e.g. on one stream.  Asynchronous; in-place
 * (d_z == d_v) is allowed. */
#define SMR_STATIC_SCRATCH_BYTES (64ull << 20)
smr_status smr_apply_P_inv_static(const smr_plan *plan, const double *d_v, double *d_z, void *stream);

/* Preconditioned MINRES on Y T x = Y b (b = the unpermuted f_H, n*m device).  d_x0: the
 * initial guess (n*m device, read only, may equal d_x) or NULL for x0 = 0, the choice of
 * the paper's experiments (Sec. 5), which also skips transforming a guess.  d_x (n*m, not
 * d_b) receives the iterate.  Stops at the first iteration whose true relative residual
 * ||b - T x||/||b|| <= rtol (rtol > 0), or after maxit (>= 0) iterations.  info_host (host)
 * receives the count and residuals.  Returns the solve status (SMR_OK on convergence).
 * Synchronises. */
smr_status smr_minres_solve(const smr_plan *plan, const double *d_b, const double *d_x0, double *d_x,
                            double rtol, int32_t maxit, smr_info *info_host, void *stream);

/* Device workspace (bytes, 256-byte aligned) that smr_minres_solve_batched needs for this
 * set of plans: the per-instance descriptor tables and status array of the batched launches. */
smr_status smr_batch_workspace_size(int32_t count, const smr_plan *const *plans, size_t *bytes);

/* The same solve for `count` independent plans at once, each with its own (N, n, scheme,
 * coefficient, preconditioner) and right-hand side.  Instances that take the sine-basis path
 * iterate together: every MINRES iteration is one per-level matvec launch per (N + 1, pprec)
 * over all variable-coefficient instances, then one fused launch per (time-size class, pprec)
 * covering all column tiles, each instance with its own device scalars; converged instances
 * are masked on the device.  The remaining instances are solved one after another on the
 * general path.  plans, d_b, d_x and infos_host are host
 * arrays of length count; d_x0 is a host array of length count or NULL (every x0 = 0);
 * d_b[i] / d_x0[i] / d_x[i] follow the conventions of smr_minres_solve.
 * d_ws: caller-owned device workspace of smr_batch_workspace_size bytes.  Every instance
 * iterates in its own plan's workspace, so a plan may appear only once per call (SMR_EINVAL
 * otherwise, before any work is enqueued).  Returns SMR_OK when every instance converged,
 * else the first failing status (each info holds its own). */
smr_status smr_minres_solve_batched(int32_t count, const smr_plan *const *plans,
                                    const double *const *d_b, const double *const *d_x0,
                                    double *const *d_x, double rtol, int32_t maxit, void *d_ws,
                                    size_t ws_bytes, smr_info *infos_host, void *stream);

/* Adjoint solve T^T lambda = g: since T^T = Y T Y, MINRES on (Y T) mu = g with the same
 * preconditioner from mu0 = 0, then lambda = Y mu.  d_g, d_lambda: n*m, distinct. */
smr_status smr_solve_adjoint(const smr_plan *plan, const double *d_g, double *d_lambda,
                             double rtol, int32_t maxit, smr_info *info_host, void *stream);

/* Batched adjoint solves T_i^T lambda_i = g_i for `count` plans (same flip-solve-flip as
 * smr_solve_adjoint, iterating together like smr_minres_solve_batched; same workspace; each
 * plan at most once). */
smr_status smr_solve_adjoint_batched(int32_t count, const smr_plan *const *plans,
                                     const double *const *d_g, double *const *d_lambda, double rtol,
                                     int32_t maxit, void *d_ws, size_t ws_bytes, smr_info *infos_host,
                                     void *stream);

/* Adjoint of smr_build_rhs (theta scheme): d_grad_f[(n+1)*m] with
 * grad f^(k) = theta tau lambda_k + (1-theta) tau lambda_{k+1} (lambda_0 = lambda_{n+1} = 0)
 * and d_grad_u0[m] = (I - (1-theta) tau K) lambda_1 (may be NULL). */
smr_status smr_rhs_adjoint(const smr_plan *plan, const double *d_lambda, double *d_grad_f,
                           double *d_grad_u0, void *stream);

/* Gradient of a loss w.r.t. the coefficient (dim 1 and 2; SMR_EUNSUPPORTED in 3D), given
 * the forward solution u (n*m), the initial value u0 (m, NULL = 0) and the adjoint
 * lambda (n*m):
 * grad a_e = -(tau/h^2) sum_k (D_e lambda_k)(D_e utilde_k), utilde_k = theta u_k + (1-theta) u_{k-1}
 * (u_0 = u0; BDF-l: utilde_k = u_k), D_e the difference across face e.  Outputs (device,
 * each may be NULL): face gradients d_gax (shaped like ax), d_gay (dim 2) and the nodal
 * gradient d_ga_nodal ((N+2)^dim, half the sum over the faces touching each node). */
smr_status smr_grad_a(const smr_plan *plan, const double *d_u, const double *d_u0,
                      const double *d_lambda, double *d_gax, double *d_gay, double *d_ga_nodal,
                      void *stream);

/* Tracing: per-kernel timing with HIP events recorded on the launch stream immediately
 * before and after every launch of a kernel class while enabled.  Classes:
 * 0 = time-axis sine transform (MFMA), 1 = spatial sine transform, 2 = space-time
 * stencil (matvec / residual), 3 = vector updates and dots, 4 = MINRES scalar steps,
 * 5 = fused sine-basis MINRES iteration, 6 = per-time-level sine-basis matvec of a variable
 * coefficient.  Launches that a solve enqueues past its
 * convergence (they exit on the device status word) are not recorded.
 * smr_profile_enable(1) clears the records and starts recording, (0) stops it.
 * smr_profile_read synchronises the recorded events and returns the launch count and
 * the summed kernel time (ms) of one class.  Not thread-safe; for diagnostics. */
smr_status smr_profile_enable(int32_t on);
smr_status smr_profile_read(int32_t kernel_class, int32_t *launches, double *total_ms);

/* Library identification and the last error message (host). */
const char *smr_version(void);
const char *smr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMR_H */
