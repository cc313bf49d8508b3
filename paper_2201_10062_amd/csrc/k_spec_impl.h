// Fused MINRES iteration in the spatial sine basis: the kernel templates, shared by the
// translation units that instantiate them for 3 time taps (theta method, BDF2) and for 5
// (BDF3, BDF4).  Included by k_spec.hip and k_spec5.hip only.
#pragma once

#include "smr_internal.h"
#include "mfma_tiles.h"

#include <algorithm>
#include <type_traits>

namespace smr {

namespace {

constexpr int kThreads = 512;         // 8 waves

constexpr int kWaves = kThreads / 64;
constexpr int kUS = 4;                // levels per batch of loads in the w/x stream
constexpr int kUA = 8;                // levels per batch of loads in the v stream

// MODE_EARLY: a steady iteration of launch 2 or 3, where w_{j-2} or w_{j-3} does not exist yet
enum { MODE_INIT = 0, MODE_FIRST = 1, MODE_STEADY = 2, MODE_EARLY = 3 };

// per-column stencil coefficients of (T y)_t = sum_k l_k y_{t-k}, k < TAPS: the time
// coefficients of the scheme plus tau mu (the column's eigenvalue) on the levels K acts on
// (theta: l_0 = 1 + theta tm, l_1 = -1 + (1 - theta) tm; BDF-l: l_0 = alpha_0 + tm,
// l_k = alpha_k)
template <int TAPS>
struct Coef {
  double l[TAPS];
};
template <int TAPS>
__device__ __forceinline__ Coef<TAPS> coef_of(const SpecP &P, double tm) {
  double tc[5], kb[2];
  (void)scheme_coefs(P.scheme, P.theta, tc, kb);
  Coef<TAPS> c;
#pragma unroll
  for (int k = 0; k < TAPS; ++k) c.l[k] = tc[k] + (k < 2 ? kb[k] * tm : 0.0);
  return c;
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

// tc: the 4 coefficients per time mode (from LDS where the block holds a copy)
__device__ __forceinline__ double inv_sigma(const double *tc, int tmode, double t) {
  const double *c = tc + 4 * tmode;
  const double re = c[0] + t * c[1];
  const double im = c[2] + t * c[3];
  return rsqrt64(re * re + im * im);
}

// A block-uniform float64 moved to scalar registers (keeps the vector registers for the
// matrix-core accumulators and the streaming carries).
__device__ __forceinline__ double uni(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sums of four values over the block, in a fixed order; the result is valid in thread 0.
// LEAD: wait first for every thread to be done reading red (not needed when barriers have
// passed since its last use).
template <int NV, bool LEAD>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*red)[kWaves]) {
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  if (LEAD) __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < kWaves; ++w) s += red[q][w];
      v[q] = s;
    }
}

// MINRES scalar recurrence after launch j-1, whose mode was pmode, from the block sums of
// that launch (run by thread 0 of every block of launch j).
// have_res = false: the true residual of the newest iterate was not evaluated (its lower
// bound excluded convergence), so only the iteration limit is tested.
__device__ void scalar_update(Scal *sc, int pmode, double s0, double s1, double s2, double s3, bool have_res) {
  if (pmode == MODE_INIT) {
    // s0 = ||v_1||^2, s1 = ||b||^2, s2 = gamma_1^2, s3 = <T^ z_1, z_1>
    sc->bnorm = sqrt(s1);
    sc->iter = 0;
    sc->nres = 1;
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
  if (pmode == MODE_STEADY) {
    if (have_res) {
      sc->nres += 1;
      sc->relres = sqrt(s0) / sc->bnorm;          // of x_{j-1}
      if (sc->relres <= sc->rtol) { sc->iter -= 1; sc->status = DONE_CONV; return; }
    }
    if (sc->exact) { sc->iter -= 1; sc->status = DONE_CONV; return; }
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

template <int HP, int C, int MODE, int PR, int TAPS>
__device__ __forceinline__ void spec_body(const SpecP &P, const int jph, const int pmode, const int tile) {
  typedef typename Prec<PR>::T T;
  typedef typename Prec<PR>::Acc Acc;
  constexpr int LD = C + 1;
  constexpr int RT = HP / 16, CT = C / 16, RPW = (RT + 3) / 4;
  constexpr int G = kThreads / C;          // row groups when all 8 waves stream
  constexpr int G2 = (kThreads / 2) / C;   // row groups of the 4 streaming waves
  extern __shared__ double lds_raw[];
  T *U = reinterpret_cast<T *>(lds_raw);   // [HP][LD]
  T *D = U + HP * LD;                      // [HP][LD]
  __shared__ double red[5][kWaves];
  __shared__ Scal S;
  // the sigma coefficients of all time modes in LDS (8 KB at hp = 128; read by the 1/sigma
  // pass); larger hp keeps reading them from L2 so that two blocks still fit per CU
  constexpr bool TCL = HP <= 128;
  __shared__ double tcs[TCL ? 8 * HP : 1];
  if (TCL)
    for (int e = threadIdx.x; e < 4 * P.n; e += kThreads) tcs[e] = P.tcoef[e];
  const double *tcl = TCL ? tcs : P.tcoef;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = P.n, m = P.m, ld = P.ld, h1 = P.h1, h2 = P.h2;
  const int col0 = tile * C;
  const int j = jph;   // launch index modulo 6 (rotation phase); INIT uses the j = 0 slots

  // ---- 0. the scalars of this launch: every block reduces the partial sums of launch j-1 (in
  //         the same fixed order, so all blocks agree bit for bit) and steps the recurrence;
  //         the block of tile 0 publishes the new state.  Scalar states and partial sums
  //         alternate between two slots by launch parity.
  if (MODE != MODE_INIT) {
    const Scal *sprev = P.sc + ((j + 1) & 1);
    if (sprev->status != RUNNING) {             // stopped earlier: pass the state on
      if (tile == 0 && tid == 0) P.sc[j & 1] = *sprev;
      return;
    }
  }
  const T *__restrict__ zcur = reinterpret_cast<const T *>(P.Z[(j + 2) % 3]);
  const T *__restrict__ zprev = reinterpret_cast<const T *>(P.Z[(j + 1) % 3]);
  T *__restrict__ znext = reinterpret_cast<T *>(MODE == MODE_INIT ? P.Z[0] : P.Z[j % 3]);
  const double *__restrict__ vcur = P.V[j % 2];
  double *__restrict__ vold = MODE == MODE_INIT ? P.V[1] : P.V[(j + 1) % 2];
  const double *__restrict__ wa = P.W[j % 2];
  double *__restrict__ wb = P.W[(j + 1) % 2];
  const double *__restrict__ bh = P.bh;
  double *__restrict__ xv = P.x;
  constexpr bool STEADY = MODE == MODE_STEADY || MODE == MODE_EARLY;

  // the v stream's column and levels (phase A), and its first batch of loads, issued before
  // the scalar step so that they are in flight during it (they do not depend on the scalars)
  const int ac = tid % C, ag = tid / C;
  const bool aok = col0 + ac < m;
  const int acc_c = aok ? col0 + ac : m - 1;         // clamped column for loads
  const int aR = (n + G - 1) / G;
  const int at0 = min(n, ag * aR), at1 = min(n, at0 + aR);   // groups past n: no level, no carry
  const bool aext = P.qext != nullptr;               // (T z)^ given by the per-level matvec
  const bool axz = MODE == MODE_INIT && P.x0zero;    // x0 = 0: no x read, (T x0)^ = 0
  auto asrc = [&](size_t i) -> double { return MODE == MODE_INIT ? (axz ? 0.0 : xv[i]) : (double)zcur[i]; };
  double ys[kUA], qs[kUA], vc[kUA], vo[kUA], bs[kUA];
  auto a_load = [&](int tb) {
#pragma unroll
    for (int u = 0; u < kUA; ++u) {
      const int t = min(tb + u, at1 - 1);            // past at1: a valid level, value unused
      const size_t it = vat(ld, t, acc_c), io = vat(ld, n - 1 - t, acc_c);
      ys[u] = aext ? 0.0 : asrc(it);
      qs[u] = aext && !axz ? P.qext[it] : 0.0;
      vc[u] = MODE == MODE_INIT ? 0.0 : vcur[io];
      vo[u] = STEADY ? vold[io] : 0.0;
      bs[u] = MODE == MODE_INIT ? bh[it] : 0.0;
    }
  };
  if (at0 < at1) a_load(at0);

  if (MODE != MODE_INIT) {
    const Scal *sprev = P.sc + ((j + 1) & 1);
    Scal *snew = P.sc + (j & 1);
    if (tid == 0) S = *sprev;      // in flight with the partial sums below
    // the previous launch's partials: one entry per tile, or per tile group once reduced
    const int npp = P.rtiles ? P.rtiles : P.tiles;
    const double *pp = P.rtiles ? P.part + 8 * (size_t)P.tiles + (size_t)((j + 1) & 1) * 4 * P.rtiles
                                : P.part + (size_t)((j + 1) & 1) * 4 * P.tiles;
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // t[4]: residuals skipped by the per-level matvec
    for (int b = tid; b < npp; b += kThreads) {
#pragma unroll
      for (int q = 0; q < 4; ++q) t[q] += pp[4 * (size_t)b + q];
    }
    if (P.qext) {           // the per-level matvec's residual and delta partials
      for (int b = tid; b < P.nks; b += kThreads) {
        const double *kp = P.kpart + 4 * (size_t)b;
        t[0] += kp[0];
        t[4] += kp[1];
        t[3] += kp[3];
      }
    }
    block_sum<5, false>(t, red);
    if (tid == 0) {
      // slot 1 of a steady launch flags a skipped residual (it holds ||b||^2 after INIT)
      scalar_update(&S, pmode, t[0], t[1], t[2], t[3], t[4] == 0.0 && (pmode != MODE_STEADY || t[1] == 0.0));
      if (tile == 0) *snew = S;
    }
    __syncthreads();
    if (S.status != RUNNING) return;
  }
  if (MODE == MODE_INIT && tile == 0 && tid == 0) {   // the state the first launch starts from
    Scal s0{};
    s0.rtol = P.rtol;
    s0.maxit = P.maxit;
    s0.status = RUNNING;
    P.sc[0] = s0;
  }
  const double va = uni(S.va), vb = uni(S.vb), zs = uni(S.zs);
  const double a1 = uni(S.a1), a2 = uni(S.a2), a3 = uni(S.a3), ceta = uni(S.ceta), zsl = uni(S.gamma_new);

  double acc_r = 0.0, acc_b = 0.0, acc_g = 0.0, acc_d = 0.0;
  // the true residual of x_{j-1} is needed only once sqrt(min sigma) |eta| (a lower bound of
  // ||r||_2, |eta| being ||r||_{P^-1}) no longer excludes convergence, or at the iteration limit
  const bool bres = STEADY && !P.qext &&
                    (P.sqsigmin * fabs(S.eta) <= 2.0 * S.rtol * S.bnorm || S.iter >= S.maxit);
  if (STEADY && !P.qext && !bres && tid == 0) acc_b = 1.0;

  // ---- B (steady launches, streaming waves 4..7): lagged w_{j-1}, x_{j-1} and the true
  //      residual of x_{j-1}, streamed over time levels with x carried for the stencil.  Each
  //      group's levels are split between the four matrix-core passes.  The carries read the
  //      previous group's last levels, so they are taken here, before any wave writes w or x.
  const bool bwave = STEADY && wave >= 4;
  const int bc = (tid - kThreads / 2) % C, bg = (tid - kThreads / 2) / C;
  const bool bok = col0 + bc < m;
  const int bcc = bok ? col0 + bc : m - 1;
  const int bR = (n + G2 - 1) / G2;
  const int bt0 = bwave ? min(n, bg * bR) : 0, bt1 = bwave ? min(n, bt0 + bR) : 0;
  int bq[5];                                   // B's levels split in four, one per GEMM pass
#pragma unroll
  for (int q = 0; q <= 4; ++q) bq[q] = bt0 + ((bt1 - bt0) * q + 3) / 4;
  // w_{j-2} exists from launch 3 on, w_{j-3} from launch 4 on (launch j has iter = j - 1);
  // in launches 2 and 3 the missing ones are read from v_j (finite) with a zero coefficient
  const bool w2 = MODE != MODE_EARLY || S.iter >= 2, w3 = MODE != MODE_EARLY || S.iter >= 3;
  const double *__restrict__ war = w2 ? wa : vcur;
  const double *__restrict__ wbr = w3 ? (const double *)wb : vcur;
  const double a2e = w2 ? a2 : 0.0, a3e = w3 ? a3 : 0.0;
  const double ra1 = 1.0 / a1;   // one division per launch instead of one per element
  auto wnew = [&](size_t i) { return (zsl * (double)zprev[i] - a3e * wbr[i] - a2e * war[i]) * ra1; };
  double bx[TAPS - 1];                          // x_{t-1}, x_{t-2}, ... (updated)
#pragma unroll
  for (int q = 0; q < TAPS - 1; ++q) {
    bx[q] = 0.0;
    if (bwave && bt0 >= q + 1) { const size_t i = vat(ld, bt0 - 1 - q, bcc); bx[q] = xv[i] + ceta * wnew(i); }
  }
  // kUS levels at a time, all their loads issued before any store (see the v stream below;
  // w_{j-1} overwrites w_{j-3} in place, each element read before it is written)
  auto bstream_t = [&](auto res, int ta, int tb) {
    constexpr bool RES = decltype(res)::value;
    const Coef<TAPS> k = coef_of<TAPS>(P, P.tmu[bcc]);
    for (int t0 = ta; t0 < tb; t0 += kUS) {
      double zp[kUS], w3[kUS], w2[kUS], xo[kUS], bt[kUS];
#pragma unroll
      for (int u = 0; u < kUS; ++u) {
        const size_t i = vat(ld, min(t0 + u, tb - 1), bcc);   // past tb: valid, unused
        zp[u] = (double)zprev[i];
        w3[u] = wbr[i];
        w2[u] = war[i];
        xo[u] = xv[i];
        bt[u] = RES ? bh[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kUS; ++u) {
        if (t0 + u >= tb) break;
        const size_t i = vat(ld, t0 + u, bcc);
        const double w = (zsl * zp[u] - a3e * w3[u] - a2e * w2[u]) * ra1;
        const double x0 = xo[u] + ceta * w;
        if (bok) {
          wb[i] = w;
          xv[i] = x0;
          if (RES) {      // (variable a: the per-level matvec takes the true residual)
            double tx = k.l[0] * x0;
#pragma unroll
            for (int q = 0; q < TAPS - 1; ++q) tx += k.l[q + 1] * bx[q];
            const double r = bt[u] - tx;
            acc_r += r * r;
          }
        }
#pragma unroll
        for (int q = TAPS - 2; q > 0; --q) bx[q] = bx[q - 1];
        bx[0] = x0;
      }
    }
  };
  auto bstream = [&](int ta, int tb) {
    if (bres) bstream_t(std::true_type{}, ta, tb);
    else bstream_t(std::false_type{}, ta, tb);
  };

  // ---- A. v_{j+1}[o] (or v_1), o = n-1-t, streamed over time levels t in ascending order
  //        so that the stencil's previous level is a register carry.  LDS mirror layout:
  //        U[o] for o < h1, D[t] for o >= h1 (so that U[p] pairs with D[p] = row n-1-p).
  {
    const int c = ac, cc = acc_c, t0 = at0, t1 = at1;
    const bool ok = aok, ext = aext, xz = axz;
    const Coef<TAPS> k = coef_of<TAPS>(P, P.tmu[cc]);
    double yc[TAPS - 1];                       // y_{t-1}, y_{t-2}, ...
#pragma unroll
    for (int q = 0; q < TAPS - 1; ++q) yc[q] = (!ext && t0 >= q + 1) ? asrc(vat(ld, t0 - 1 - q, cc)) : 0.0;
    // kUA levels at a time, all their loads issued before any store (the stores of one level
    // would otherwise hold back the loads of the next: the compiler cannot separate them);
    // the first batch was loaded before the scalar step
    for (int tb = t0; tb < t1; tb += kUA) {
      if (tb != t0) a_load(tb);
#pragma unroll
      for (int u = 0; u < kUA; ++u) {
        const int t = tb + u;
        if (t >= t1) break;
        const int o = n - 1 - t;
        const size_t it = vat(ld, t, cc), io = vat(ld, o, cc);
        const double y0 = ys[u];
        double st = k.l[0] * y0;
#pragma unroll
        for (int q = 0; q < TAPS - 1; ++q) st += k.l[q + 1] * yc[q];
        const double ty = ext ? qs[u] : st;
        double v;
        if (MODE == MODE_INIT) {
          v = bs[u] - ty;                              // (Y b)_o - ((Y T)^ x0)_o
          if (ok) { acc_r += v * v; acc_b += bs[u] * bs[u]; }
          if (xz && ok) xv[it] = 0.0;
        } else if (MODE == MODE_FIRST) {
          v = zs * ty - va * vc[u];                    // v_0 = 0
        } else {
          v = zs * ty - va * vc[u] - vb * vo[u];
        }
        if (ok) vold[io] = v;
        if (o < h1) U[o * LD + c] = ok ? (T)v : T(0);
        else D[t * LD + c] = ok ? (T)v : T(0);
#pragma unroll
        for (int q = TAPS - 2; q > 0; --q) yc[q] = yc[q - 1];
        yc[0] = y0;
      }
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

  // ---- C. the matrix-core waves: z = S_o^T D_o S_o u | S_e^T D_e S_e d, one table per pass
  //         (each result goes back to LDS once every wave is done reading that block); the
  //         streaming waves run a quarter of B beside each pass.
  Acc acc[RPW][CT];
  const T *So = reinterpret_cast<const T *>(P.So), *Se = reinterpret_cast<const T *>(P.Se);
  const T *SoT = reinterpret_cast<const T *>(P.SoT), *SeT = reinterpret_cast<const T *>(P.SeT);
  if (wave < 4) gemm_tiles<HP, C, PR>(So, U, wave, lane, acc);
  else if (STEADY) bstream(bq[0], bq[1]);
  __syncthreads();
  if (wave < 4) {
    store_acc<HP, C, PR>(acc, U, wave, lane);     // S_o u -> U
    gemm_tiles<HP, C, PR>(Se, D, wave, lane, acc);
  } else if (STEADY) {
    bstream(bq[1], bq[2]);
  }
  __syncthreads();
  if (wave < 4) store_acc<HP, C, PR>(acc, D, wave, lane);   // S_e d -> D
  __syncthreads();
  // scale by 1/sigma (time mode 2p+1 is row p of U, mode 2p+2 row p of D) and the Parseval
  // partial of gamma^2, all waves; rows past h1 / h2 and columns past m stay zero
  for (int e = tid; e < HP * C; e += kThreads) {
    const int pp = e / C, cl = e - pp * C, col = col0 + cl;
    const bool okc = col < m;
    const double tm = P.tmu[okc ? col : m - 1];
    double so = 0.0, se = 0.0;
    if (okc && pp < h1) {
      const double a = (double)U[pp * LD + cl];
      so = a * inv_sigma(tcl, 2 * pp, tm);
      acc_g += a * so;
    }
    if (okc && pp < h2) {
      const double a = (double)D[pp * LD + cl];
      se = a * inv_sigma(tcl, 2 * pp + 1, tm);
      acc_g += a * se;
    }
    U[pp * LD + cl] = (T)so;
    D[pp * LD + cl] = (T)se;
  }
  __syncthreads();
  if (wave < 4) gemm_tiles<HP, C, PR>(SoT, U, wave, lane, acc);
  else if (STEADY) bstream(bq[2], bq[3]);
  __syncthreads();
  if (wave < 4) {
    store_acc<HP, C, PR>(acc, U, wave, lane);     // u' -> U
    gemm_tiles<HP, C, PR>(SeT, D, wave, lane, acc);
  } else if (STEADY) {
    bstream(bq[3], bq[4]);
  }
  __syncthreads();
  if (wave < 4) store_acc<HP, C, PR>(acc, D, wave, lane);   // d' -> D
  __syncthreads();

  // ---- D. store z_{j+1} and accumulate <(Y T)^ z, z> = sum_t (T z)_t z_{n-1-t}
  {
    const int c = tid % C, g = tid / C;
    const int col = col0 + c;
    const bool ok = col < m;
    const Coef<TAPS> k = coef_of<TAPS>(P, P.tmu[ok ? col : m - 1]);
    const int R = (n + G - 1) / G;
    const int t0 = min(n, g * R), t1 = min(n, t0 + R);   // groups past n take no level
    // z_p = u'_p + d'_p and z_{n-1-p} = u'_p - d'_p (p < h2); odd n: the middle z_p = u'_p
    auto zrow = [&](int t) -> double {
      if (t < h1) return t < h2 ? (double)(T)(U[t * LD + c] + D[t * LD + c]) : (double)U[t * LD + c];
      const int p = n - 1 - t;
      return (double)(T)(U[p * LD + c] - D[p * LD + c]);
    };
    double yc[TAPS - 1];
#pragma unroll
    for (int q = 0; q < TAPS - 1; ++q) yc[q] = t0 >= q + 1 ? zrow(t0 - 1 - q) : 0.0;
#pragma unroll 2
    for (int t = t0; t < t1; ++t) {
      const double y0 = zrow(t);
      if (ok) {
        znext[vat(ld, t, col)] = (T)y0;
        if (!P.qext) {
          double ty = k.l[0] * y0;
#pragma unroll
          for (int q = 0; q < TAPS - 1; ++q) ty += k.l[q + 1] * yc[q];
          acc_d += ty * zrow(n - 1 - t);
        }
      }
#pragma unroll
      for (int q = TAPS - 2; q > 0; --q) yc[q] = yc[q - 1];
      yc[0] = y0;
    }
  }

  // ---- E. block partials of this launch (reduced at the start of the next one)
  double t[4] = {acc_r, acc_b, acc_g, acc_d};
  block_sum<4, false>(t, red);
  if (tid == 0) {
    double *pp = P.part + (size_t)(j & 1) * 4 * P.tiles + 4 * (size_t)tile;
    pp[0] = t[0]; pp[1] = t[1]; pp[2] = t[2]; pp[3] = t[3];
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin in block order.  Give each XCD a
// contiguous range of tiles instead, so that neighbouring tiles run side by side under the
// same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  constexpr int kXcd = 8;
  const int x = bid % kXcd, local = bid / kXcd;
  const int per = nb / kXcd, rem = nb % kXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

template <int HP, int C, int MODE, int PR, int TAPS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HP >= 256 ? 2 : 4, 8)))
void k_spec(SpecP P, int jph, int pmode) {
  spec_body<HP, C, MODE, PR, TAPS>(P, jph, pmode, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched launch: the blocks of every instance in the table, instance found by its first block.
template <int HP, int C, int MODE, int PR, int TAPS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HP >= 256 ? 2 : 4, 8)))
void k_spec_multi(const SpecP *__restrict__ table, int ninst, int jph, int pmode) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].tile0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const SpecP &P = table[lo];   // read in place (a private copy would go to scratch)
  spec_body<HP, C, MODE, PR, TAPS>(P, jph, pmode, b - P.tile0);
}

template <int HP, int C, int PR, int TAPS>
hipError_t run_spec(hipStream_t st, const SpecP &P, int mode, int blocks, int jph, int pmode) {
  const size_t shmem = 2 * (size_t)HP * (C + 1) * sizeof(typename Prec<PR>::T);
  if (shmem > 65536) {
    (void)lds_limit((const void *)k_spec<HP, C, 0, PR, TAPS>, shmem);
    (void)lds_limit((const void *)k_spec<HP, C, 1, PR, TAPS>, shmem);
    (void)lds_limit((const void *)k_spec<HP, C, 2, PR, TAPS>, shmem);
    (void)lds_limit((const void *)k_spec<HP, C, 3, PR, TAPS>, shmem);
  }
  if (mode == 0) hipLaunchKernelGGL((k_spec<HP, C, 0, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, P, jph, pmode);
  else if (mode == 1) hipLaunchKernelGGL((k_spec<HP, C, 1, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, P, jph, pmode);
  else if (mode == 2) hipLaunchKernelGGL((k_spec<HP, C, 2, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, P, jph, pmode);
  else hipLaunchKernelGGL((k_spec<HP, C, 3, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, P, jph, pmode);
  return hipGetLastError();
}

template <int HP, int C, int PR, int TAPS>
hipError_t run_spec_multi(hipStream_t st, const SpecP *table, int ninst, int mode, int blocks, int jph, int pmode) {
  const size_t shmem = 2 * (size_t)HP * (C + 1) * sizeof(typename Prec<PR>::T);
  if (shmem > 65536) {
    (void)lds_limit((const void *)k_spec_multi<HP, C, 0, PR, TAPS>, shmem);
    (void)lds_limit((const void *)k_spec_multi<HP, C, 1, PR, TAPS>, shmem);
    (void)lds_limit((const void *)k_spec_multi<HP, C, 2, PR, TAPS>, shmem);
    (void)lds_limit((const void *)k_spec_multi<HP, C, 3, PR, TAPS>, shmem);
  }
  if (mode == 0)
    hipLaunchKernelGGL((k_spec_multi<HP, C, 0, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph, pmode);
  else if (mode == 1)
    hipLaunchKernelGGL((k_spec_multi<HP, C, 1, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph, pmode);
  else if (mode == 2)
    hipLaunchKernelGGL((k_spec_multi<HP, C, 2, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph, pmode);
  else
    hipLaunchKernelGGL((k_spec_multi<HP, C, 3, PR, TAPS>), dim3(blocks), dim3(kThreads), shmem, st, table, ninst, jph, pmode);
  return hipGetLastError();
}

template <int PR, int C, int TAPS>
hipError_t run_spec_hp(hipStream_t st, const SpecP &P, int mode, int blocks, int hp, int jph, int pmode) {
  switch (hp) {
    case 16: return run_spec<16, C, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    case 32: return run_spec<32, C, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    case 64: return run_spec<64, C, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    case 128: return run_spec<128, C, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    default: break;
  }
  if constexpr (C == 16) {   // two 32-column LDS blocks of 256 or more rows do not fit
    if (hp == 256) return run_spec<256, 16, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    if (hp == 512) return run_spec<512, 16, PR, TAPS>(st, P, mode, blocks, jph, pmode);
  }
  return hipErrorInvalidValue;
}

template <int PR, int C, int TAPS>
hipError_t run_multi_hp(hipStream_t st, const SpecP *table, int ninst, int mode, int blocks, int hp, int jph,
                        int pmode) {
  switch (hp) {
    case 16: return run_spec_multi<16, C, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    case 32: return run_spec_multi<32, C, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    case 64: return run_spec_multi<64, C, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    case 128: return run_spec_multi<128, C, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    default: break;
  }
  if constexpr (C == 16) {
    if (hp == 256) return run_spec_multi<256, 16, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    if (hp == 512) return run_spec_multi<512, 16, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
  }
  return hipErrorInvalidValue;
}

// 64-column tiles (hp <= 64, or 128 with float32 transforms: fewer blocks pay the fixed costs)
template <int PR, int TAPS>
hipError_t run_spec_hp64(hipStream_t st, const SpecP &P, int mode, int blocks, int hp, int jph, int pmode) {
  switch (hp) {
    case 16: return run_spec<16, 64, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    case 32: return run_spec<32, 64, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    case 64: return run_spec<64, 64, PR, TAPS>(st, P, mode, blocks, jph, pmode);
    default: break;
  }
  if constexpr (PR == 1)
    if (hp == 128) return run_spec<128, 64, 1, TAPS>(st, P, mode, blocks, jph, pmode);
  return hipErrorInvalidValue;
}
template <int PR, int TAPS>
hipError_t run_multi_hp64(hipStream_t st, const SpecP *table, int ninst, int mode, int blocks, int hp, int jph,
                          int pmode) {
  switch (hp) {
    case 16: return run_spec_multi<16, 64, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    case 32: return run_spec_multi<32, 64, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    case 64: return run_spec_multi<64, 64, PR, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
    default: break;
  }
  if constexpr (PR == 1)
    if (hp == 128) return run_spec_multi<128, 64, 1, TAPS>(st, table, ninst, mode, blocks, jph, pmode);
  return hipErrorInvalidValue;
}

// One launch of the fused kernel (single plan) or of its batched variant, dispatched on the
// transform precision, the column-tile width and the time padding.
template <int TAPS>
hipError_t run_one_taps(hipStream_t st, const SpecP &P, int pprec, int cols, int mode, int blocks, int hp, int jph,
                        int pmode) {
  if (cols == 64)
    return pprec == SMR_FP32 ? run_spec_hp64<1, TAPS>(st, P, mode, blocks, hp, jph, pmode)
                             : run_spec_hp64<0, TAPS>(st, P, mode, blocks, hp, jph, pmode);
  if (cols == 16)
    return pprec == SMR_FP32 ? run_spec_hp<1, 16, TAPS>(st, P, mode, blocks, hp, jph, pmode)
                             : run_spec_hp<0, 16, TAPS>(st, P, mode, blocks, hp, jph, pmode);
  if (cols == 32)
    return pprec == SMR_FP32 ? run_spec_hp<1, 32, TAPS>(st, P, mode, blocks, hp, jph, pmode)
                             : run_spec_hp<0, 32, TAPS>(st, P, mode, blocks, hp, jph, pmode);
  return hipErrorInvalidValue;
}

template <int TAPS>
hipError_t run_multi_taps(hipStream_t st, const SpecP *table, int ninst, int blocks, int hp, int cols, int pprec,
                          int mode, int jph, int pmode) {
  if (cols == 64)
    return pprec == SMR_FP32 ? run_multi_hp64<1, TAPS>(st, table, ninst, mode, blocks, hp, jph, pmode)
                             : run_multi_hp64<0, TAPS>(st, table, ninst, mode, blocks, hp, jph, pmode);
  if (cols == 16)
    return pprec == SMR_FP32 ? run_multi_hp<1, 16, TAPS>(st, table, ninst, mode, blocks, hp, jph, pmode)
                             : run_multi_hp<0, 16, TAPS>(st, table, ninst, mode, blocks, hp, jph, pmode);
  if (cols == 32)
    return pprec == SMR_FP32 ? run_multi_hp<1, 32, TAPS>(st, table, ninst, mode, blocks, hp, jph, pmode)
                             : run_multi_hp<0, 32, TAPS>(st, table, ninst, mode, blocks, hp, jph, pmode);
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace smr
