// Fused MINRES iteration in the spatial sine basis (gfx950), for constant coefficients.
//
// When a is constant, K = U Lambda U with U the (orthogonal, symmetric) spatial sine
// transform (Sec. 3.1.1), and both Y T and P_H / Phat are block diagonal over the
// spatial modes after the change of basis I (x) U:
//   (Y T)^ : per spatial mode k a flipped time stencil l0_k z_t + l1_k z_{t-1} (+ l2 z_{t-2});
//   P^-1 ^ : per spatial mode k the time-axis S_n diag(1/sigma_{.,k}) S_n.
// MINRES is invariant under an orthogonal change of basis, so the iteration runs on the
// transformed vectors and only b, x0 and the result cross the spatial transform.  One
// kernel does a whole iteration for a tile of C spatial modes (all n time levels):
//   A. q = (Y T)^ zt_j, v_{j+1} = q - va v_j - vb v_{j-1} (stored), butterflied into LDS;
//      lagged search direction w_{j-1} and x_{j-1} (its coefficients need gamma_j, which
//      the previous launch produced);
//   B. true residual of x_{j-1}: ||Y b - (Y T)^ x||^2 partial;
//   C. z_{j+1} = S diag(1/sigma) S v_{j+1} on the FP64 matrix cores (two folded GEMMs),
//      gamma_{j+1}^2 = <v, z> by Parseval between them;
//   D. z_{j+1} stored, <(Y T)^ z_{j+1}, z_{j+1}> partial (gives delta_{j+1});
//   E. block partials -> the last block to finish reduces them in a fixed order and runs
//      the MINRES scalar recurrence (Givens rotation, convergence test).
// The iterate x_{j-1} and its residual are final one launch after v_j, z_j: the stop test
// is the same (first iteration whose true residual is <= rtol), one launch later.
#include "smr_internal.h"

#include <type_traits>

namespace smr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 512;         // 8 waves

// Arithmetic of the time transform: PR 0 = float64 (v_mfma_f64_16x16x4f64), PR 1 = float32
// (v_mfma_f32_16x16x4f32).  Fragment layouts (checked on gfx950): A[i][k] in lane i + 16k and
// B[k][j] in lane j + 16k for both; accumulator register r of lane l holds D[4r + l/16][l%16]
// for float64 but D[4(l/16) + r][l%16] for float32.
template <int PR> struct Prec;
template <> struct Prec<0> {
  typedef double T;
  typedef d4 Acc;
  static __device__ __forceinline__ Acc mfma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int bk) { return 4 * q + bk; }
};
template <> struct Prec<1> {
  typedef float T;
  typedef f4 Acc;
  static __device__ __forceinline__ Acc mfma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int bk) { return 4 * bk + q; }
};
constexpr int kWaves = kThreads / 64;

enum { MODE_INIT = 0, MODE_FIRST = 1, MODE_STEADY = 2 };

// per-column stencil coefficients of (T y)_t = l0 y_t + l1 y_{t-1} + l2 y_{t-2}
struct Coef {
  double l0, l1, l2;
};
__device__ __forceinline__ Coef coef_of(const SpecP &P, double tm) {
  if (P.scheme == SMR_THETA) return Coef{1.0 + P.theta * tm, -1.0 + (1.0 - P.theta) * tm, 0.0};
  return Coef{1.5 + tm, -2.0, 0.5};
}

// Sine-basis vectors are (n, ld) row-major with the row stride ld a multiple of 32, so a
// 32-mode column tile covers whole 256-byte (float64) or 128-byte (float32) lines per level.
__device__ __forceinline__ size_t vat(int ld, int t, int q) { return (size_t)t * ld + q; }

// 1/|re + i im| from a float reciprocal square root refined by two Newton steps in float64
// (relative error ~1e-16, well inside the 1e-12 parity bound of the preconditioner).
__device__ __forceinline__ double rsqrt64(double q) {
  double r = (double)__frsqrt_rn((float)q);
  r = r * (1.5 - 0.5 * q * r * r);
  r = r * (1.5 - 0.5 * q * r * r);
  return r;
}

__device__ __forceinline__ double inv_sigma(const SpecP &P, int tmode, double t) {
  const double *c = P.tcoef + 4 * tmode;
  const double re = c[0] + t * c[1];
  const double im = c[2] + t * c[3];
  return rsqrt64(re * re + im * im);
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kWaves; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double ld_agent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// MINRES scalar recurrence for one launch (thread 0 of the last block).
template <int MODE>
__device__ void scalar_update(Scal *sc, double s0, double s1, double s2, double s3) {
  if (MODE == MODE_INIT) {
    // s0 = ||v_1||^2, s1 = ||b||^2, s2 = gamma_1^2, s3 = <T^ z_1, z_1>
    sc->bnorm = sqrt(s1);
    sc->iter = 0;
    sc->exact = 0;
    sc->status = RUNNING;
    if (s1 == 0.0) { sc->relres = 0.0; sc->status = DONE_CONV; return; }
    sc->relres = sqrt(s0) / sc->bnorm;
    if (sc->relres <= sc->rtol) { sc->status = DONE_CONV; return; }
    if (!(s2 > 0.0) || !isfinite(s2)) { sc->status = DONE_NOTSPD; return; }
    if (sc->maxit <= 0) { sc->status = DONE_MAXIT; return; }
    const double g = sqrt(s2);
    sc->gamma = g; sc->gamma1 = g; sc->gamma_old = 1.0;
    sc->eta = g; sc->c = sc->c_old = 1.0; sc->s = sc->s_old = 0.0;
    sc->delta = s3 / s2;
    sc->zs = 1.0 / g;
    sc->va = sc->delta / g;
    sc->vb = 0.0;
    return;
  }
  // s0 = ||r(x_{j-1})||^2 (STEADY), s2 = gamma_{j+1}^2, s3 = <T^ z_{j+1}, z_{j+1}>
  sc->iter += 1;                                  // launches since INIT = j
  if (MODE == MODE_STEADY) {
    sc->relres = sqrt(s0) / sc->bnorm;            // of x_{j-1}
    if (sc->relres <= sc->rtol || sc->exact) { sc->iter -= 1; sc->status = DONE_CONV; return; }
    if (sc->iter - 1 >= sc->maxit) { sc->iter -= 1; sc->status = DONE_MAXIT; return; }
  }
  if (s2 < 0.0 || !isfinite(s2)) { sc->iter -= 1; sc->status = DONE_NOTSPD; return; }
  const double gn = sqrt(s2);
  const double g = sc->gamma, dl = sc->delta;
  const double a0 = sc->c * dl - sc->c_old * sc->s * g;
  const double a1 = sqrt(a0 * a0 + gn * gn);
  const double a2 = sc->s * dl + sc->c_old * sc->c * g;
  const double a3 = sc->s_old * g;
  if (a1 == 0.0) { sc->iter -= 1; sc->status = DONE_BREAKDOWN; return; }
  sc->c_old = sc->c; sc->c = a0 / a1;
  sc->s_old = sc->s; sc->s = gn / a1;
  sc->a1 = a1; sc->a2 = a2; sc->a3 = a3;
  sc->ceta = sc->c * sc->eta;
  sc->eta = -sc->s * sc->eta;
  sc->gamma_new = sc->zs;                         // 1/gamma_j for the lagged w_j (next launch)
  sc->gamma_old = g;
  sc->gamma = gn;
  if (gn == 0.0) {                                // Krylov space exhausted: x_j is exact
    sc->exact = 1;
    sc->delta = 0.0; sc->va = 0.0; sc->vb = 0.0; sc->zs = 0.0;
  } else {
    sc->delta = s3 / s2;
    sc->va = sc->delta / gn;
    sc->vb = gn / g;
    sc->zs = 1.0 / gn;
  }
}

// GEMM of the four matrix-core waves: for the 16-row tiles r = wave + 4 i (i < RPW) and all
// CT column tiles, ao[i][ct] += A_o[r] * U[:, ct] and ae[i][ct] += A_e[r] * D[:, ct] over the
// k dimension.  One A fragment feeds CT MFMAs.  The tables hold the fragments of k-steps
// 2q and 2q+1 side by side per lane, so one load fetches two k-steps; loads run two such
// pairs (four k-steps) ahead of the matrix cores.
template <int HP, int C, int PR>
__device__ __forceinline__ void gemm_tiles(const typename Prec<PR>::T *__restrict__ Ao,
                                           const typename Prec<PR>::T *__restrict__ Ae,
                                           const typename Prec<PR>::T *U, const typename Prec<PR>::T *D,
                                           int wave, int lane,
                                           typename Prec<PR>::Acc (&ao)[(HP / 16 + 3) / 4][C / 16],
                                           typename Prec<PR>::Acc (&ae)[(HP / 16 + 3) / 4][C / 16]) {
  typedef typename Prec<PR>::T T;
  typedef typename std::conditional<PR == 0, double2, float2>::type T2;
  constexpr int LD = C + 1;
  constexpr int RT = HP / 16, CT = C / 16, RPW = (RT + 3) / 4;
  constexpr int KS = HP / 4, KP = KS / 2;         // k-steps, k-step pairs
  const int bk = lane >> 4, bj = lane & 15;
  const T2 *__restrict__ Ao2 = reinterpret_cast<const T2 *>(Ao);
  const T2 *__restrict__ Ae2 = reinterpret_cast<const T2 *>(Ae);
  const T2 zero2 = {T(0), T(0)};
  T2 q0u[RPW], q0d[RPW], q1u[RPW], q1d[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wave + 4 * i;
    const size_t base = (size_t)r * KP * 64 + lane;
    const bool ok = r < RT;
    q0u[i] = ok ? Ao2[base] : zero2;
    q0d[i] = ok ? Ae2[base] : zero2;
    q1u[i] = (ok && KP > 1) ? Ao2[base + 64] : zero2;
    q1d[i] = (ok && KP > 1) ? Ae2[base + 64] : zero2;
  }
  for (int kp = 0; kp < KP; ++kp) {
    T2 q2u[RPW], q2d[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + 4 * i;
      const bool more = r < RT && kp + 2 < KP;
      const size_t at = ((size_t)r * KP + kp + 2) * 64 + lane;
      q2u[i] = more ? Ao2[at] : zero2;
      q2d[i] = more ? Ae2[at] : zero2;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = 2 * kp + h;
      T bu[CT], bd[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        bu[ct] = U[(4 * kk + bk) * LD + 16 * ct + bj];
        bd[ct] = D[(4 * kk + bk) * LD + 16 * ct + bj];
      }
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        if (wave + 4 * i < RT) {
          const T au = h ? q0u[i].y : q0u[i].x;
          const T ad = h ? q0d[i].y : q0d[i].x;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            ao[i][ct] = Prec<PR>::mfma(au, bu[ct], ao[i][ct]);
            ae[i][ct] = Prec<PR>::mfma(ad, bd[ct], ae[i][ct]);
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      q0u[i] = q1u[i]; q0d[i] = q1d[i];
      q1u[i] = q2u[i]; q1d[i] = q2d[i];
    }
  }
}

template <int HP, int C, int MODE, int PR>
__device__ __forceinline__ void spec_body(const SpecP &P, const int jph, const int tile) {
  typedef typename Prec<PR>::T T;
  typedef typename Prec<PR>::Acc Acc;
  Scal *sc = P.sc;
  if (MODE != MODE_INIT && sc->status != RUNNING) return;
  constexpr int LD = C + 1;
  constexpr int RT = HP / 16, CT = C / 16, RPW = (RT + 3) / 4;
  constexpr int G = kThreads / C;          // row groups when all 8 waves stream
  constexpr int G2 = (kThreads / 2) / C;   // row groups of the 4 streaming waves
  extern __shared__ double lds_raw[];
  T *U = reinterpret_cast<T *>(lds_raw);   // [HP][LD]
  T *D = U + HP * LD;                      // [HP][LD]
  __shared__ double red[kWaves];
  __shared__ int is_last;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = P.n, m = P.m, ld = P.ld, h1 = P.h1, h2 = P.h2;
  const int col0 = tile * C;
  const double va = sc->va, vb = sc->vb, zs = sc->zs;
  const double a1 = sc->a1, a2 = sc->a2, a3 = sc->a3, ceta = sc->ceta, zsl = sc->gamma_new;
  const int j = jph;   // launch index modulo 6 (rotation phase); INIT uses the j = 0 slots
  const T *__restrict__ zcur = reinterpret_cast<const T *>(P.Z[(j + 2) % 3]);
  const T *__restrict__ zprev = reinterpret_cast<const T *>(P.Z[(j + 1) % 3]);
  T *__restrict__ znext = reinterpret_cast<T *>(MODE == MODE_INIT ? P.Z[0] : P.Z[j % 3]);
  const double *__restrict__ vcur = P.V[j % 2];
  double *__restrict__ vold = MODE == MODE_INIT ? P.V[1] : P.V[(j + 1) % 2];
  const double *__restrict__ wa = P.W[j % 2];
  double *__restrict__ wb = P.W[(j + 1) % 2];
  const double *__restrict__ bh = P.bh;
  double *__restrict__ xv = P.x;

  double acc_r = 0.0, acc_b = 0.0, acc_g = 0.0, acc_d = 0.0;

  // ---- B (steady launches, streaming waves 4..7): lagged w_{j-1}, x_{j-1} and the true
  //      residual of x_{j-1}, streamed over time levels with x carried for the stencil.  Each
  //      group's levels are split between the two matrix-core windows.  The carries read the
  //      previous group's last levels, so they are taken here, before any wave writes w or x.
  const bool bwave = MODE == MODE_STEADY && wave >= 4;
  const int bc = (tid - kThreads / 2) % C, bg = (tid - kThreads / 2) / C;
  const bool bok = col0 + bc < m;
  const int bcc = bok ? col0 + bc : m - 1;
  const int bR = (n + G2 - 1) / G2;
  const int bt0 = bwave ? min(n, bg * bR) : 0, bt1 = bwave ? min(n, bt0 + bR) : 0;
  const int bmid = bt0 + (bt1 - bt0 + 1) / 2;
  auto wnew = [&](size_t i) { return (zsl * (double)zprev[i] - a3 * wb[i] - a2 * wa[i]) / a1; };
  double bx1 = 0.0, bx2 = 0.0;
  if (bwave) {
    if (bt0 >= 1) { const size_t i = vat(ld, bt0 - 1, bcc); bx1 = xv[i] + ceta * wnew(i); }
    if (bt0 >= 2) { const size_t i = vat(ld, bt0 - 2, bcc); bx2 = xv[i] + ceta * wnew(i); }
  }
  auto bstream = [&](int ta, int tb) {
    const Coef k = coef_of(P, P.tmu[bcc]);
#pragma unroll 4
    for (int t = ta; t < tb; ++t) {
      const size_t i = vat(ld, t, bcc);
      const double w = wnew(i);
      const double x0 = xv[i] + ceta * w;
      const double r = bh[i] - (k.l0 * x0 + k.l1 * bx1 + k.l2 * bx2);
      if (bok) {
        wb[i] = w;
        xv[i] = x0;
        acc_r += r * r;
      }
      bx2 = bx1;
      bx1 = x0;
    }
  };

  // ---- A. v_{j+1}[o] (or v_1), o = n-1-t, streamed over time levels t in ascending order
  //        so that the stencil's previous level is a register carry.  LDS mirror layout:
  //        U[o] for o < h1, D[t] for o >= h1 (so that U[p] pairs with D[p] = row n-1-p).
  {
    const int c = tid % C, g = tid / C;
    const int col = col0 + c;
    const bool ok = col < m;
    const int cc = ok ? col : m - 1;                 // clamped column for loads
    const Coef k = coef_of(P, P.tmu[cc]);
    const int R = (n + G - 1) / G;
    const int t0 = g * R, t1 = min(n, t0 + R);
    auto src = [&](size_t i) -> double { return MODE == MODE_INIT ? xv[i] : (double)zcur[i]; };
    double y1 = t0 >= 1 ? src(vat(ld, t0 - 1, cc)) : 0.0;
    double y2 = t0 >= 2 ? src(vat(ld, t0 - 2, cc)) : 0.0;
#pragma unroll 4
    for (int t = t0; t < t1; ++t) {
      const int o = n - 1 - t;
      const size_t it = vat(ld, t, cc), io = vat(ld, o, cc);
      const double y0 = src(it);
      const double ty = k.l0 * y0 + k.l1 * y1 + k.l2 * y2;
      double v;
      if (MODE == MODE_INIT) {
        const double bt = bh[it];
        v = bt - ty;                                 // (Y b)_o - ((Y T)^ x0)_o
        if (ok) { acc_r += v * v; acc_b += bt * bt; }
      } else {
        v = zs * ty - va * vcur[io] - vb * vold[io];
      }
      if (ok) vold[io] = v;
      if (o < h1) U[o * LD + c] = ok ? (T)v : T(0);
      else D[t * LD + c] = ok ? (T)v : T(0);
      y2 = y1;
      y1 = y0;
    }
    // padding rows
    for (int e = tid; e < (HP - h1) * C; e += kThreads) U[(h1 + e / C) * LD + e % C] = T(0);
    for (int e = tid; e < (HP - h2) * C; e += kThreads) D[(h2 + e / C) * LD + e % C] = T(0);
  }
  __syncthreads();
  // butterfly in place: (U[p], D[p]) <- (v_p + v_{n-1-p}, v_p - v_{n-1-p}); odd n: middle has d = 0
  for (int e = tid; e < h1 * C; e += kThreads) {
    const int pp = e / C, c = e % C;
    const T a = U[pp * LD + c];
    const T b = pp < h2 ? D[pp * LD + c] : T(0);
    U[pp * LD + c] = pp < h2 ? a + b : a;
    if (pp < h2) D[pp * LD + c] = a - b;
  }
  __syncthreads();

  Acc ao[RPW][CT], ae[RPW][CT];
  const Acc zacc = {0, 0, 0, 0};
  const T *So = reinterpret_cast<const T *>(P.So), *Se = reinterpret_cast<const T *>(P.Se);
  const T *SoT = reinterpret_cast<const T *>(P.SoT), *SeT = reinterpret_cast<const T *>(P.SeT);
  if (wave < 4) {
    // ---- C. the matrix-core waves: z = S_o^T D_o S_o u | S_e^T D_e S_e d
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) { ao[i][ct] = zacc; ae[i][ct] = zacc; }
    gemm_tiles<HP, C, PR>(So, Se, U, D, wave, lane, ao, ae);
  } else if (MODE == MODE_STEADY) {
    bstream(bt0, bmid);   // B, first half of each group's levels
  }
  __syncthreads();   // matrix-core waves are done reading U, D
  if (wave < 4) {
    // scale by 1/sigma (time mode 2p+1 -> index 2p, 2p+2 -> 2p+1), Parseval partial
    const int bk = lane >> 4, bj = lane & 15;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + 4 * i;
      if (r >= RT) continue;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int cl = 16 * ct + bj, col = col0 + cl;
        const double tm = P.tmu[col < m ? col : m - 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pp = 16 * r + Prec<PR>::row(q, bk);
          double so = 0.0, se = 0.0;
          if (col < m && pp < h1) {
            const double a = (double)ao[i][ct][q];
            so = a * inv_sigma(P, 2 * pp, tm);
            acc_g += a * so;
          }
          if (col < m && pp < h2) {
            const double a = (double)ae[i][ct][q];
            se = a * inv_sigma(P, 2 * pp + 1, tm);
            acc_g += a * se;
          }
          U[pp * LD + cl] = (T)so;
          D[pp * LD + cl] = (T)se;
        }
      }
    }
  }
  __syncthreads();
  if (wave < 4) {
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) { ao[i][ct] = zacc; ae[i][ct] = zacc; }
    gemm_tiles<HP, C, PR>(SoT, SeT, U, D, wave, lane, ao, ae);
  } else if (MODE == MODE_STEADY) {
    bstream(bmid, bt1);   // B, second half
  }
  __syncthreads();   // U, D free again
  if (wave < 4) {
    // z_p = u'_p + d'_p -> U[p]; z_{n-1-p} = u'_p - d'_p -> D[p]; odd n: middle z_p = u'_p
    const int bk = lane >> 4, bj = lane & 15;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + 4 * i;
      if (r >= RT) continue;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int cl = 16 * ct + bj;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pp = 16 * r + Prec<PR>::row(q, bk);
          if (pp < h2) {
            U[pp * LD + cl] = ao[i][ct][q] + ae[i][ct][q];
            D[pp * LD + cl] = ao[i][ct][q] - ae[i][ct][q];
          } else if (pp < h1) {
            U[pp * LD + cl] = ao[i][ct][q];
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- D. store z_{j+1} and accumulate <(Y T)^ z, z> = sum_t (T z)_t z_{n-1-t}
  {
    const int c = tid % C, g = tid / C;
    const int col = col0 + c;
    const bool ok = col < m;
    const Coef k = coef_of(P, P.tmu[ok ? col : m - 1]);
    const int R = (n + G - 1) / G;
    const int t0 = g * R, t1 = min(n, t0 + R);
    auto zrow = [&](int t) -> double { return (double)(t < h1 ? U[t * LD + c] : D[(n - 1 - t) * LD + c]); };
    double y1 = t0 >= 1 ? zrow(t0 - 1) : 0.0;
    double y2 = t0 >= 2 ? zrow(t0 - 2) : 0.0;
#pragma unroll 4
    for (int t = t0; t < t1; ++t) {
      const double y0 = zrow(t);
      if (ok) {
        znext[vat(ld, t, col)] = (T)y0;
        acc_d += (k.l0 * y0 + k.l1 * y1 + k.l2 * y2) * zrow(n - 1 - t);
      }
      y2 = y1;
      y1 = y0;
    }
  }

  // ---- E. block partials, last block reduces in a fixed order and steps the scalars
  const double s0 = block_sum(acc_r, red);
  const double s1 = block_sum(acc_b, red);
  const double s2 = block_sum(acc_g, red);
  const double s3 = block_sum(acc_d, red);
  if (tid == 0) {
    double *pp = P.part + 4 * (size_t)tile;
    pp[0] = s0; pp[1] = s1; pp[2] = s2; pp[3] = s3;
    __threadfence();
    const int ticket = atomicAdd(P.counter, 1);
    is_last = (ticket == P.tiles - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
  for (int b = tid; b < P.tiles; b += kThreads) {
    const double *pp = P.part + 4 * (size_t)b;
    t0 += ld_agent(pp + 0);
    t1 += ld_agent(pp + 1);
    t2 += ld_agent(pp + 2);
    t3 += ld_agent(pp + 3);
  }
  t0 = block_sum(t0, red);
  t1 = block_sum(t1, red);
  t2 = block_sum(t2, red);
  t3 = block_sum(t3, red);
  if (tid == 0) {
    scalar_update<MODE>(sc, t0, t1, t2, t3);
    *P.counter = 0;
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin in block order.  Give each XCD a
// contiguous range of tiles instead, so that the tiles sharing a cache line at a row-segment
// boundary (rows of m doubles are not line aligned) run side by side under the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  constexpr int kXcd = 8;
  const int x = bid % kXcd, local = bid / kXcd;
  const int per = nb / kXcd, rem = nb % kXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

template <int HP, int C, int MODE, int PR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HP >= 256 ? 2 : 4, 8)))
void k_spec(SpecP P, int jph) {
  spec_body<HP, C, MODE, PR>(P, jph, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched launch: the blocks of every instance in the table, instance found by its first block.
template <int HP, int C, int MODE, int PR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HP >= 256 ? 2 : 4, 8)))
void k_spec_multi(const SpecP *__restrict__ table, int ninst, int jph) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].tile0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const SpecP P = table[lo];
  spec_body<HP, C, MODE, PR>(P, jph, b - P.tile0);
}

template <int HP, int C, int PR>
hipError_t run_spec(hipStream_t st, const SpecP &P, int mode, int blocks, int jph) {
  const size_t shmem = 2 * (size_t)HP * (C + 1) * sizeof(typename Prec<PR>::T);
  if (shmem > 65536) {
    hipFuncSetAttribute((const void *)k_spec<HP, C, 0, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    hipFuncSetAttribute((const void *)k_spec<HP, C, 1, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    hipFuncSetAttribute((const void *)k_spec<HP, C, 2, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  }
  if (mode == 0) hipLaunchKernelGGL((k_spec<HP, C, 0, PR>), dim3(blocks), dim3(kThreads), shmem, st, P, jph);
  else if (mode == 1) hipLaunchKernelGGL((k_spec<HP, C, 1, PR>), dim3(blocks), dim3(kThreads), shmem, st, P, jph);
  else hipLaunchKernelGGL((k_spec<HP, C, 2, PR>), dim3(blocks), dim3(kThreads), shmem, st, P, jph);
  return hipGetLastError();
}

template <int HP, int C, int PR>
hipError_t run_spec_multi(hipStream_t st, const SpecP *table, int ninst, int mode, int blocks, int jph) {
  const size_t shmem = 2 * (size_t)HP * (C + 1) * sizeof(typename Prec<PR>::T);
  if (shmem > 65536) {
    hipFuncSetAttribute((const void *)k_spec_multi<HP, C, 0, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    hipFuncSetAttribute((const void *)k_spec_multi<HP, C, 1, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    hipFuncSetAttribute((const void *)k_spec_multi<HP, C, 2, PR>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  }
  if (mode == 0)
    hipLaunchKernelGGL((k_spec_multi<HP, C, 0, PR>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph);
  else if (mode == 1)
    hipLaunchKernelGGL((k_spec_multi<HP, C, 1, PR>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph);
  else
    hipLaunchKernelGGL((k_spec_multi<HP, C, 2, PR>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph);
  return hipGetLastError();
}

template <int PR>
hipError_t run_spec_hp(hipStream_t st, const SpecP &P, int mode, int blocks, int hp, int jph) {
  switch (hp) {
    case 16: return run_spec<16, 32, PR>(st, P, mode, blocks, jph);
    case 32: return run_spec<32, 32, PR>(st, P, mode, blocks, jph);
    case 64: return run_spec<64, 32, PR>(st, P, mode, blocks, jph);
    case 128: return run_spec<128, 32, PR>(st, P, mode, blocks, jph);
    case 256: return run_spec<256, 16, PR>(st, P, mode, blocks, jph);
    case 512: return run_spec<512, 16, PR>(st, P, mode, blocks, jph);
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int PR>
hipError_t run_multi_hp(hipStream_t st, const SpecP *table, int ninst, int mode, int blocks, int hp, int jph) {
  switch (hp) {
    case 16: return run_spec_multi<16, 32, PR>(st, table, ninst, mode, blocks, jph);
    case 32: return run_spec_multi<32, 32, PR>(st, table, ninst, mode, blocks, jph);
    case 64: return run_spec_multi<64, 32, PR>(st, table, ninst, mode, blocks, jph);
    case 128: return run_spec_multi<128, 32, PR>(st, table, ninst, mode, blocks, jph);
    case 256: return run_spec_multi<256, 16, PR>(st, table, ninst, mode, blocks, jph);
    case 512: return run_spec_multi<512, 16, PR>(st, table, ninst, mode, blocks, jph);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

int spec_cols(const Plan *p) { return p->hp >= 256 ? 16 : 32; }

int spec_blocks(const Plan *p) {
  const int C = spec_cols(p);
  return (p->m + C - 1) / C;
}

SpecP spec_desc(const Plan *p, double *x, const double *bh) {
  SpecP P{};
  P.n = p->n; P.m = p->m; P.ld = p->ld; P.h1 = p->h1; P.h2 = p->h2; P.scheme = p->scheme; P.theta = p->theta;
  P.tiles = spec_blocks(p);
  P.tile0 = 0;
  const bool f32 = p->pprec == SMR_FP32;
  P.So = f32 ? (const void *)p->Sof : (const void *)p->So;
  P.SoT = f32 ? (const void *)p->SoTf : (const void *)p->SoT;
  P.Se = f32 ? (const void *)p->Sef : (const void *)p->Se;
  P.SeT = f32 ? (const void *)p->SeTf : (const void *)p->SeT;
  P.tcoef = p->tcoef; P.tmu = p->tmu;
  for (int i = 0; i < 3; ++i) P.Z[i] = f32 ? (void *)p->ZF[i] : (void *)(i == 0 ? p->Z[0] : i == 1 ? p->Z[1] : p->Q);
  P.V[0] = p->V[0]; P.V[1] = p->V[1]; P.W[0] = p->W[0]; P.W[1] = p->W[1];
  P.x = x; P.bh = bh; P.part = p->part; P.counter = p->counter; P.sc = p->sc;
  return P;
}

hipError_t launch_spec(Ctx c, int mode, int j, double *x, const double *bh) {
  const Plan *p = c.p;
  const SpecP P = spec_desc(p, x, bh);
  const int jph = j % 6;
  return p->pprec == SMR_FP32 ? run_spec_hp<1>(c.st, P, mode, P.tiles, p->hp, jph)
                              : run_spec_hp<0>(c.st, P, mode, P.tiles, p->hp, jph);
}

hipError_t launch_spec_multi(hipStream_t st, const SpecP *table, int ninst, int blocks, int hp, int pprec, int mode,
                             int j) {
  const int jph = j % 6;
  return pprec == SMR_FP32 ? run_multi_hp<1>(st, table, ninst, mode, blocks, hp, jph)
                           : run_multi_hp<0>(st, table, ninst, mode, blocks, hp, jph);
}

__global__ void k_gather_scal(const SpecP *__restrict__ table, int ninst, Scal *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) out[i] = *table[i].sc;
}

hipError_t launch_gather_scal(hipStream_t st, const SpecP *table, int ninst, Scal *out) {
  hipLaunchKernelGGL(k_gather_scal, dim3((ninst + 63) / 64), dim3(64), 0, st, table, ninst, out);
  return hipGetLastError();
}

}  // namespace smr
