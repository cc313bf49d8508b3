// Internal declarations shared by the host driver and the HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "smr.h"

namespace smr {

constexpr int kMaxN = 511;       // N + 1 <= 512
constexpr int kMaxN3 = 127;      // N + 1 <= 128 in 3D (the stencil's spatial tiles fit the partial slots)
constexpr int kMaxn = 1024;
constexpr int kRedSlots = 8192;  // partial sums per reduction (grid-stride kernels use <= this many blocks)
constexpr size_t kKsPartOffset = 8 * (size_t)kRedSlots;   // per-level partials of the sine-basis matvec
constexpr int kKsTiles = 8;      // row / column tiles per level of the tiled N = 127 matvec (16 lines each)
// Above this many column tiles, a fused launch's partial sums are first reduced by kPartGroups
// blocks (one fixed group of tiles each) instead of being re-read in full by every block of
// the next launch.
constexpr int kDirectTiles = 1024;
constexpr int kPartGroups = 64;

// MINRES status codes kept on the device.
enum DevStatus : int { RUNNING = 0, DONE_CONV = 1, DONE_MAXIT = 2, DONE_NOTSPD = 3, DONE_BREAKDOWN = 4 };

// Device-resident MINRES scalars of one instance (Paige-Saunders recurrence).
struct Scal {
  double gamma, gamma_old, gamma_new;   // Lanczos normalisers
  double delta;                         // <A zt, zt>
  double c, c_old, s, s_old;            // the two latest Givens rotations
  double eta;                           // rotated residual (|eta| = P^{-1}-norm residual)
  double gamma1, bnorm;                 // initial gamma and ||rhs||_2
  double a1, a2, a3, ceta;              // search-direction coefficients of the current step
  double relres;                        // latest true relative residual
  double zs;                            // 1/gamma for the current z
  double va, vb;                        // v_{j+1} = q - va v_j - vb v_{j-1}
  double rtol;
  int iter, status, maxit, exact;
  int nres, pad;                        // true residuals evaluated so far
};

// Time coefficients of one block row of T (Sec. 1 and Sec. 4): (T x)_t = sum_k c_k x_{t-k} +
// tau K (b_0 x_t + b_1 x_{t-1}).  Theta method: c = (1, -1), b = (theta, 1 - theta); BDF-l: c
// the l-step backward difference formula (sum_{j=1}^{l} nabla^j / j), b = (1, 0).  Returns the
// number of levels (2, or l + 1); c is zero past it.  Shared by the host set-up and the kernels,
// which take the scheme and theta from their descriptors rather than a coefficient array.
__host__ __device__ inline int scheme_coefs(int scheme, double theta, double (&c)[5], double (&b)[2]) {
  for (int k = 0; k < 5; ++k) c[k] = 0.0;
  b[0] = 1.0;
  b[1] = 0.0;
  switch (scheme) {
    case SMR_BDF2: c[0] = 1.5; c[1] = -2.0; c[2] = 0.5; return 3;
    case SMR_BDF3: c[0] = 11.0 / 6.0; c[1] = -3.0; c[2] = 1.5; c[3] = -1.0 / 3.0; return 4;
    case SMR_BDF4: c[0] = 25.0 / 12.0; c[1] = -4.0; c[2] = 3.0; c[3] = -4.0 / 3.0; c[4] = 0.25; return 5;
    default: c[0] = 1.0; c[1] = -1.0; b[0] = theta; b[1] = 1.0 - theta; return 2;
  }
}

// Host-side plan: parameters plus device pointers into the caller's workspace.
struct Plan {
  // parameters
  int dim, N, n, m, scheme, precond, pprec, cheb_k, flags;
  int taps;                   // time levels one block row of T couples: 2 (theta), l + 1 (BDF-l)
  double tcf[5];              // time-difference coefficients of those levels (theta: 1, -1;
                              // BDF-l: alpha_0 .. alpha_l), zero past taps
  double kbf[2];              // weights of K on levels t and t-1 (theta: theta, 1 - theta; BDF: 1, 0)
  size_t len;                 // n*m
  int ld;                     // row stride of the sine-basis vectors: m rounded up to 32
  size_t vlen;                // n*ld: elements of every work vector
  double T, tau, theta, h, h2inv;
  bool const_coef;            // every face value equal
  double a_min, a_max, abar, cheb_lo, cheb_hi;
  double kbar_d, kbar_cx, kbar_cy, kbar_cz;
  double sqsigmin;            // sqrt of the smallest eigenvalue of P (P_H / Phat)
  int L, logL;                // L = N + 1 = 2^logL (spatial sine transform length)
  int h1, h2, hp;             // folded time halves: ceil(n/2), floor(n/2), padded to 16
  int spec_c;                 // column-tile width of the fused sine-basis kernel (16 or 32)
  int pinv_var;               // physical-basis P^{-1}: 0 float64 intermediates, 1 float32, 2 float32
                              // with 16-line column tiles, 3 float64 with 16-line column tiles
                              // (float32 only in SMR_FP32 solves); -1 on the sine-basis path
  // tables (device)
  double *ax, *ay, *az;       // face values (filled with 1 for a = 1; az in 3D only)
  double *tmu;                // m: tau * eigenvalue of K (a const) or Kbar, sine-basis order
  double *tmu_lap;            // m: tau * eigenvalue of the a = 1 Laplacian
  double *tcoef;              // 4*hp*2: per time mode (A, B, C, D) of sigma, grouped by parity
  double *ez;                 // 2n: eta_j, zeta_j (P_theta)
  double *So, *SoT, *Se, *SeT;  // folded time sine blocks in MFMA fragment order (hp*hp)
  float *Sof, *SoTf, *Sef, *SeTf;  // the same in float32 (mixed precision)
  double *tw;                 // complex twiddles exp(-2 pi i t / (2L)), t < L (interleaved)
  // vectors (device), each vlen doubles (physical-basis use: stride m; sine basis: stride ld)
  double *V[2], *Z[2], *W[2], *Q, *T1, *T2, *T3, *T4, *G;
  double *QX;                 // (T z)^ of the variable-coefficient sine-basis solve (or null)
  double *Y[4];               // level intermediates of the tiled N = 127 matvec (or null)
  bool ks_split;              // N = 127 matvec as three passes over line tiles, not one level per block
  double *gface;              // 2 (N+1)^2 face-gradient scratch
  float *ZF[3];               // float32 z vectors of the mixed-precision sine-basis solve
  double *part;               // >= 16 * kRedSlots partial sums (more when the fused kernel's
                              // column tiles need them)
  Scal *sc;                   // device scalars (2 slots; the physical-basis path uses slot 0)
  // host-side resources of the sine-basis solve, made on first use, released by smr_destroy
  mutable hipGraphExec_t steady6 = nullptr;          // six captured steady iterations
  mutable Scal *snap = nullptr;                      // two pinned host status snapshots
  mutable hipEvent_t snap_ev[2] = {nullptr, nullptr};
  mutable hipStream_t cap = nullptr;                 // stream the steady graph is captured on
  Scal *sc_host;              // pinned host mirror
  size_t ws_bytes;
};

// ---------------------------------------------------------------- launchers
// All launch on `st` and return hipSuccess or the launch error.
struct Ctx {
  const Plan *p;
  hipStream_t st;
};

// Raises a kernel's dynamic LDS limit to `bytes` on the current device, calling the runtime
// only the first time (per kernel, device and larger size) instead of on every launch.
hipError_t lds_limit(const void *kernel, size_t bytes);

// y = Y T (xs * x) with xs = *d_xscale (or 1 if null); optional partial sums of
// y . (xs*x) into part[0..G).  When rhs != null computes r = Y rhs - Y T x instead and
// accumulates ||r||^2 (slot 0) and ||rhs||^2 (slot 1) and writes r if y != null.
hipError_t launch_apply_YT(Ctx c, const double *x, const double *d_xscale, double *y,
                           const double *rhs, double *part, int *nblocks_out, const Scal *gate);
hipError_t launch_build_rhs(Ctx c, const double *f, const double *u0, double *b);
hipError_t launch_rhs_adjoint(Ctx c, const double *lam, double *gf, double *gu0);
hipError_t launch_grad_faces(Ctx c, const double *u, const double *u0, const double *lam,
                             double *gax, double *gay, double *gnodal);

// Spatial sine transform (orthonormal DST-I) along x (dir 0), y (dir 1) or z (dir 2, 3D) of nslices
// slices; in-place allowed when the strides agree.  Slice strides of in and out default
// (0) to m.  scale_mode 1 divides the result by the Chebyshev inner diagonal
// eta_s + zeta_s * abar * tau * mu_lap; scale_mode 2 (2D column pass with N + 1 = 256 only,
// else hipErrorInvalidValue) divides by it and applies the column transform once more.
hipError_t launch_dst(Ctx c, int dir, const double *in, double *out, int nslices, int scale_mode,
                      const Scal *gate, long in_stride = 0, long out_stride = 0);
// The same pass with float32 (in32 / out32) or float64 input and output vectors; the
// transform itself runs in float64 (float32 intermediates of a mixed-precision P^{-1}).
// col16: 16-line tiles in the column passes of the line-tile kernels (else 8).
hipError_t launch_dst_v(Ctx c, int dir, const void *in, bool in32, void *out, bool out32, int nslices,
                        int scale_mode, const Scal *gate, long in_stride = 0, long out_stride = 0,
                        bool col16 = false);
// The last spatial pass (rows, 2D, N + 1 = 256) of the Chebyshev inner preconditioner with the
// Chebyshev update taking its result t in place of a store: dvec = a_t t (first) or
// a_d dvec + a_t t, then x = dvec (first) or x + dvec (every vector float32 when f32).
hipError_t launch_dst_cheb_axpy(Ctx c, const void *in, void *x, void *dvec, bool f32, double a_d, double a_t,
                                int first, const Scal *gate);
// Time transform: mode 0: out = (S_n (x) I) in; mode 1: out = (S_n (x) I) diag(1/sigma) (S_n (x) I) in
// with partial sums of <D vhat, vhat> into part when part != null.  f32: the GEMMs on the
// float32 matrix cores with the plan's float32 sine tables (pprec SMR_FP32 plans only).
hipError_t launch_time(Ctx c, const double *in, double *out, int mode, double *part, int *nblocks_out,
                       const Scal *gate, bool f32 = false);
// Float32 GEMMs (SMR_FP32 plans) with float32 (in32 / out32) or float64 vectors in memory.
hipError_t launch_time_v(Ctx c, const void *in, bool in32, void *out, bool out32, int mode, double *part,
                         int *nblocks_out, const Scal *gate);

// Elementwise / reductions / scalar steps.
hipError_t launch_vupdate(Ctx c, const double *q, const double *v, double *vold_inout, const Scal *gate);
hipError_t launch_wxupdate(Ctx c, const double *z, double *wold_inout, const double *w, double *x,
                           const Scal *gate);
hipError_t launch_dot(Ctx c, const double *a, const double *b, double *part, int *nblocks_out,
                      const Scal *gate);
hipError_t launch_scale_copy(Ctx c, const double *in, double *out, double s, int flip);
hipError_t launch_zero(Ctx c, double *x, size_t len);
// stage: 0 = init (part slot0 = ||r0||^2, slot1 = ||b||^2, part2 = gamma^2 partials)
//        1 = delta, 2 = gamma_new + Givens, 3 = true residual / convergence
hipError_t launch_scalar_step(Ctx c, int stage, const double *part, int nb, const double *part2,
                              int nb2);

// Fused MINRES iteration in the spatial sine basis (constant coefficients, P_H / Phat).
// mode 0 = initialise from x0, 1 = first iteration, 2 = steady iteration; j = launch index
// (selects the rotating z / v / w buffers).  x and bh are the transformed iterate and rhs.
// One instance of the sine-basis solve as the fused kernel sees it (also the element of the
// device descriptor table of a batched launch).
struct SpecP {
  int n, m, ld, h1, h2, scheme, tiles, tile0;   // ld: row stride of the vectors below
  double theta;
  double sqsigmin;       // sqrt of the smallest eigenvalue of P (residual lower bound)
  const void *So, *SoT, *Se, *SeT;   // folded sine tables in the transform's precision
  const double *tcoef, *tmu;
  // vectors (spatial-sine basis, (n, ld) row-major); z in the transform's precision.  Launch j uses
  // z_j = Z[(j-1)%3], z_{j+1} = Z[j%3], z_{j-1} = Z[(j+1)%3], v_j = V[j%2], v_{j-1} = V[(j+1)%2]
  // (overwritten by v_{j+1}), w_{j-2} = W[j%2], w_{j-3} = W[(j+1)%2] (overwritten by w_{j-1}).
  void *Z[3];
  double *V[2], *W[2];
  double *x;             // x (INIT: x0, read only)
  const double *bh;      // transformed right-hand side b^ (unpermuted)
  double *part;          // 2 slots (launch parity) of 4 partial sums per column tile; with
                         // rtiles > 0 two further slots of 4 per tile group follow them
  Scal *sc;              // 2 scalar states: sc[j & 1] is the state after launch j
  // variable coefficient: (T z)^ comes from the per-level kernel, with its partial sums
  // [residual^2, residual skipped, 0, delta] per time level (null / 0 for constant a)
  const double *qext;
  const double *kpart;
  int nks;
  int x0zero;            // INIT: the solve starts from x0 = 0 (x is written, not read)
  double rtol;           // INIT: the starting scalar state (sc[0]) it writes
  int maxit;
  int rtiles;            // 0: a launch reads every tile's partials; else the number of tile
                         // groups whose sums a reduction launch left at part + 8 tiles
};

// One instance of the per-level sine-basis matvec (also the element of its batched table).
struct KsP {
  int N, n, m, ld, L, scheme, blk0, pad;
  double theta, tau, h2inv, scale, sqsigmin;
  const double *ax, *ay, *tw;
  const void *Z[3];      // z rotation of the fused kernel (the transform's precision)
  const double *x, *bh;  // iterate and right-hand side (sine basis)
  double *q;             // out: (T s)^
  double *kpart;         // out: 4 partial sums per time level (per level and tile when tiled)
  double *y[4];          // intermediates of the tiled N = 127 passes (source chain, residual chain)
  const Scal *sc;
};
bool kslice_supported(const Plan *p);
// 2D spatial sine transform of every time level in one pass (dim 2, N + 1 in {32, 64, 128});
// out may equal in only when the strides agree.  stop_gate: run only once that scalar state
// is no longer RUNNING (a transform enqueued ahead of a predicted stop).
hipError_t launch_dst2d(Ctx c, const double *in, double *out, long in_stride, long out_stride,
                        const Scal *stop_gate = nullptr);
// One DST-I pass (the arguments of launch_dst) as line tiles through the register FFT, for 2D
// plans with N + 1 in {32, 64, 128, 256}; launch_dst takes it where it applies.
bool dst_tile_supported(const Plan *p);
hipError_t launch_dst_tile(Ctx c, int dir, const void *in, bool in32, void *out, bool out32, int nslices, int scale_mode,
                           const Scal *gate, long in_stride, long out_stride, bool col16 = false);
KsP kslice_desc(const Plan *p, double *x, const double *bh);
// mode 0: q = (T x)^ before the initialising launch; mode 1: q = (T z_j)^ with its partials
// before fused launch j
hipError_t launch_kslice(Ctx c, int mode, int j, double *x, const double *bh);
// split: the class runs the tiled N = 127 passes (levels = blocks of the level kernel).
hipError_t launch_kslice_multi(hipStream_t st, const KsP *table, int ninst, int blocks, int L, int pprec, int mode,
                               int j, bool split = false);

// INIT (mode 0) also writes the starting scalar state (rtol, maxit) and, with x0zero, x = 0.
hipError_t launch_spec(Ctx c, int mode, int j, double *x, const double *bh, bool x0zero = false,
                       double rtol = 0.0, int maxit = 0);
// cols: column-tile width of the launch (0: the plan's own)
SpecP spec_desc(const Plan *p, double *x, const double *bh, int cols = 0);
// Doubles of partial-sum storage the fused kernel needs for a plan of m spatial modes
// (either tile width, with the grouped reduction above kDirectTiles tiles).
size_t spec_part_doubles(int m);
hipError_t launch_spec_multi(hipStream_t st, const SpecP *table, int ninst, int blocks, int hp, int cols, int pprec,
                             int taps, int mode, int j);
hipError_t launch_gather_scal(hipStream_t st, const SpecP *table, int ninst, int slot, Scal *out);
// Column-tile width (spatial modes per workgroup) of the fused kernel: 16 or 32, the latter
// for hp <= 128 only (two 32-column LDS blocks of 256 rows do not fit).
int spec_cols(const Plan *p);
int spec_cols_default(int hp);
bool spec_cols_ok(int hp, int cols, int pprec = SMR_FP64);
// Times one steady launch per width on the plan's (still empty) work vectors and stores the
// faster width in p->spec_c; synchronises st.
hipError_t spec_tune(Plan *p, hipStream_t st);
hipError_t launch_zero_int(Ctx c, int *x, int count);

// ---------------------------------------------------------------- autotuner (tune.cpp)
// Process-wide cache of timed launch choices per device, keyed by the shape they depend on.
bool tune_get(const std::vector<long> &key, int *choice);
void tune_put(const std::vector<long> &key, int choice);
void tune_stats(long *entries, long *hits, long *misses);
void tune_clear();
// One warm call of run, then reps timed calls on st (HIP events); ms per call.  Synchronises st.
hipError_t tune_time(hipStream_t st, int reps, const std::function<hipError_t()> &run, float *ms_per_call);
// Cache keys (first element) of the tuned choices.
enum TuneKind : long { TUNE_SPEC_WIDTH = 1, TUNE_PINV = 2, TUNE_BATCH_WIDTH = 3, TUNE_KSLICE = 4 };
// The scalar state and partial sums of a running steady iteration that never converges, for
// timing fused launches on a plan's workspace (k_spec.hip).
hipError_t spec_tune_state(const Plan *p, hipStream_t st, const SpecP &P);

// Chebyshev per-mode solve pieces (P_theta).
// f32: the vectors are float32 (mixed-precision P^{-1}); the arithmetic is float64 either way.
hipError_t launch_cheb_axpy(Ctx c, void *x, void *dvec, const void *tmp, double a_d, double a_t,
                            int first, const Scal *gate, bool f32 = false);
hipError_t launch_cheb_resid(Ctx c, void *res, const void *dvec, const Scal *gate, bool f32 = false);

}  // namespace smr
