// All-at-once matvec in the spatial sine basis for a variable coefficient (gfx950).
//
// With U the orthonormal 2D sine transform (symmetric, U U = I) and K(a) the 5-point
// stiffness matrix of eqn:matrix_Km_va built from face values, the blocks of T
// (Sec. 1: theta method A0 = I + theta tau K, A1 = -I + (1-theta) tau K; BDF2
// A0 = 1.5 I + tau K, A1 = -2 I, A2 = 0.5 I, Sec. 4) act on sine-basis levels z_t as
//   (T z)^_t = c0 z_t + c1 z_{t-1} + c2 z_{t-2} + tau U K(a) U (b0 z_t + b1 z_{t-1}),
// (c0, c1, c2) = (1, -1, 0), (b0, b1) = (theta, 1 - theta) for theta; (1.5, -2, 0.5), (1, 0)
// for BDF2.  For constant a the last term is diagonal and the fused iteration kernel
// applies it itself; here one block takes one time level through U, K(a), U with the
// level held in LDS, and writes q_t = (T z)^_t for the fused kernel, plus the partial sums
// that the MINRES scalars need from the matvec:
//   delta = <(Y T)^ z, z> = sum_t q_t . z_{n-1-t}, and (when asked) the true residual
//   ||b^ - (T x)^||^2 of the latest iterate x, by a second pass on x.
//
// Each 1D sine transform of two lines a, b (N = L - 1 points, L a power of two) packs
// z = a + i b, extends it oddly to M = 2L points and takes an M-point DFT in registers of
// one wave: M = R * 64, lane l holds z[64 j1 + l] (j1 < R); an R-point DFT in the lane,
// twiddles W_M^{l k1}, then a 64-point decimation-in-frequency DFT across lanes, after
// which lane l holds Z[k1 + R bitrev6(l)].  (S a)_k = -Im Z_{k+1} / sqrt(2L) and
// (S b)_k = Re Z_{k+1} / sqrt(2L).
#include "smr_internal.h"

#include <algorithm>
#include <type_traits>

namespace smr {

namespace {

constexpr int kKT = 512;                 // 8 waves per block
constexpr int kLB = 8;                   // elements per thread whose loads are issued together
constexpr int kKW = kKT / 64;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ int brev6(int l) { return (int)(__brev((unsigned)l) >> 26); }

// Workgroups go to the 8 XCDs round-robin in block order; give each XCD a contiguous range of
// tiles instead, so that the tiles sharing cache lines (column tiles of one slice) meet in the
// same L2.
__device__ __forceinline__ int xcd_block(int bid, int nb) {
  constexpr int kXcd = 8;
  const int x = bid % kXcd, local = bid / kXcd;
  const int per = nb / kXcd, rem = nb % kXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// Value of lane (lane ^ d) for spans 1, 2, 4 and 8, which stay inside a 16-lane row: DPP
// moves (quad_perm [1,0,3,2] and [2,3,0,1]; row_half_mirror then quad_perm [3,2,1,0], i.e.
// xor 7 then xor 3; row_ror:8).
template <int D>
__device__ __forceinline__ int xor_lane_i(int v) {
  static_assert(D == 1 || D == 2 || D == 4 || D == 8, "spans 16 and 32 use pair_vals");
  if (D == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  if (D == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  if (D == 4) return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
  return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
}
template <int D>
__device__ __forceinline__ double xor_lane(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = xor_lane_i<D>((int)(u & 0xffffffff)), hi = xor_lane_i<D>((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Spans 16 and 32: both values of the lane pair (l, l ^ D) on both lanes, a = the value of
// the lower lane (l & D == 0), b = that of the upper one.  gfx950's permlane swaps do this in
// registers: swapping a register with itself, rows 1 and 3 against rows 0 and 2 (span 16)
// or lanes 32-63 against lanes 0-31 (span 32), leaves the lower lanes' values in the first
// result and the upper lanes' values in the second, on every lane.
template <int D>
__device__ __forceinline__ void pair_vals(double x, double &a, double &b) {
  static_assert(D == 16 || D == 32, "spans 16 and 32 only");
  const long long u = __double_as_longlong(x);
  const unsigned lo = (unsigned)(u & 0xffffffff), hi = (unsigned)(u >> 32);
  unsigned alo, blo, ahi, bhi;
  if constexpr (D == 32) {
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    alo = rl[0]; blo = rl[1]; ahi = rh[0]; bhi = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    alo = rl[0]; blo = rl[1]; ahi = rh[0]; bhi = rh[1];
  }
  a = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
  b = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
}

// W_M^t for 0 <= t < M from the half table tw[t] = exp(-2 pi i t / M), t < M/2
__device__ __forceinline__ double2 twid(const double2 *__restrict__ tw, int t, int M) {
  const double2 w = tw[t < M / 2 ? t : t - M / 2];
  return t < M / 2 ? w : make_double2(-w.x, -w.y);
}

// Per-lane constants of the wave DFT, loaded once: in-lane twiddles W_M^{lane k1}
// (k1 = 1..R-1) and, per cross-lane stage s of span d = 32 >> s, the sign sg = +1 (lane in
// the top half of its pair) or -1 and the multiplier wm = 1 (top) or W_{2d}^{lane mod d}.
template <int R>
struct Twiddles {
  double2 in[R > 1 ? R - 1 : 1];
  double2 wm[6];
  double sg[6];
  __device__ __forceinline__ void load(const double2 *__restrict__ tw, int lane) {
    constexpr int M = 64 * R;
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) in[k1 - 1] = twid(tw, lane * k1, M);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int d = 32 >> s;
      const bool top = (lane & d) == 0;
      sg[s] = top ? 1.0 : -1.0;
      wm[s] = top ? make_double2(1.0, 0.0) : tw[(lane & (d - 1)) * (M / (2 * d))];
    }
  }
};

// One cross-lane stage of span D: all exchanges first, then per value (sg v + p) wm with p
// the partner's value (spans up to 8), or (a + sg b) wm with a, b the pair's lower and upper
// values (spans 16 and 32); both are a + b on the lower lane and a - b on the upper one.
template <int R, int D>
__device__ __forceinline__ void dif_stage(double2 (&v)[R], double sg, double2 wm) {
  double2 p[R];
  if constexpr (D >= 16) {
    double2 q[R];
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      pair_vals<D>(v[k1].x, p[k1].x, q[k1].x);
      pair_vals<D>(v[k1].y, p[k1].y, q[k1].y);
    }
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      const double tx = fma(sg, q[k1].x, p[k1].x), ty = fma(sg, q[k1].y, p[k1].y);
      v[k1] = cmul(make_double2(tx, ty), wm);
    }
  } else {
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      p[k1].x = xor_lane<D>(v[k1].x);
      p[k1].y = xor_lane<D>(v[k1].y);
    }
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      const double tx = fma(sg, v[k1].x, p[k1].x), ty = fma(sg, v[k1].y, p[k1].y);
      // span 1: the upper lane's multiplier is W_2^0 = 1, so no lane multiplies
      v[k1] = D == 1 ? make_double2(tx, ty) : cmul(make_double2(tx, ty), wm);
    }
  }
}

// In-lane 8-point DFT in natural order, v[k] <- sum_j v[j] exp(-2 pi i j k / 8): radix-2
// decimation in frequency (spans 4, 2, 1), then the bit-reversal permutation.
__device__ __forceinline__ double2 mul_w8(double2 a, int k) {   // a exp(-2 pi i k / 8)
  constexpr double h = 0.70710678118654752440;                   // cos(pi / 4)
  switch (k & 7) {
    case 0: return a;
    case 1: return make_double2(h * (a.x + a.y), h * (a.y - a.x));
    case 2: return make_double2(a.y, -a.x);
    default: return make_double2(h * (a.y - a.x), -h * (a.x + a.y));   // k = 3
  }
}
__device__ __forceinline__ void lane_dft8(double2 (&v)[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 a = v[k], c = v[k + 4];
    v[k] = cadd(a, c);
    v[k + 4] = mul_w8(csub(a, c), k);
  }
#pragma unroll
  for (int b = 0; b < 8; b += 4)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double2 a = v[b + k], c = v[b + k + 2];
      v[b + k] = cadd(a, c);
      v[b + k + 2] = mul_w8(csub(a, c), 2 * k);
    }
#pragma unroll
  for (int b = 0; b < 8; b += 2) {
    const double2 a = v[b], c = v[b + 1];
    v[b] = cadd(a, c);
    v[b + 1] = csub(a, c);
  }
  // position q holds frequency brev3(q): swap 1 <-> 4 and 3 <-> 6
  double2 t = v[1]; v[1] = v[4]; v[4] = t;
  t = v[3]; v[3] = v[6]; v[6] = t;
}

// In-register M-point DFT (M = 64 R) of the values v[j1] = z[64 j1 + lane]; on return
// v[k1] = Z[k1 + R brev6(lane)].  A decimation-in-frequency butterfly of the pair
// (a, b) = (top, bottom) gives a + b on the top lane and (a - b) w on the bottom one; with
// p the partner's value both are (sg v + p) wm, so every lane runs the same arithmetic.
// Each stage issues all of its cross-lane reads before using them.
template <int R>
__device__ __forceinline__ void wave_dft(double2 (&v)[R], int lane, const Twiddles<R> &W) {
  if (R == 2) {
    const double2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  } else if (R == 4) {
    const double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const double2 a2 = cadd(v[1], v[3]), a3 = csub(v[1], v[3]);
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = make_double2(a1.x + a3.y, a1.y - a3.x);   // a1 - i a3
    v[3] = make_double2(a1.x - a3.y, a1.y + a3.x);   // a1 + i a3
  }
  if constexpr (R == 8) lane_dft8(v);
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) v[k1] = cmul(v[k1], W.in[k1 - 1]);
  dif_stage<R, 32>(v, W.sg[0], W.wm[0]);
  dif_stage<R, 16>(v, W.sg[1], W.wm[1]);
  dif_stage<R, 8>(v, W.sg[2], W.wm[2]);
  dif_stage<R, 4>(v, W.sg[3], W.wm[3]);
  dif_stage<R, 2>(v, W.sg[4], W.wm[4]);
  dif_stage<R, 1>(v, W.sg[5], W.wm[5]);
}

// A whole N x N level in LDS (N = 32 R - 1), skewed so that the transforms' scattered stores
// spread over the banks: element (r, c) sits at r LP + (r >> 5) + c + (c >> 5), i.e. one pad
// slot after every 32 columns and after every 32 rows, with the pitch LP = 1 mod 8.  One
// store instruction of a wave's transform writes positions R b + k of a row or of a column
// (fixed k, b = brev6(lane) over the 32 lanes with an output in range); with a plain pitch
// these meet on the same banks 4 ways (R = 4) or 2 ways (R = 2) (64 banks of 4 bytes), with
// the skew every lane has banks of its own.  R = 1 stores consecutive positions and keeps the
// plain layout (pitch N + 2).
template <int R>
struct Lvl {
  static constexpr int N = 32 * R - 1;
  static constexpr bool SKEW = R > 1;
  static constexpr int CP = SKEW ? (N - 1) + ((N - 1) >> 5) + 1 : N;   // slots of a row, pads included
  static constexpr int LP = SKEW ? (CP + 6) / 8 * 8 + 1 : N + 2;       // skewed: smallest >= CP that is 1 mod 8
  static constexpr int SIZE = SKEW ? (N - 1) * LP + ((N - 1) >> 5) + CP : N * LP;
  __device__ static __forceinline__ int at(int r, int c) {
    return SKEW ? r * LP + (r >> 5) + c + (c >> 5) : r * LP + c;
  }
};

// Orthonormal DST-I of every row (DIR 0) or column (DIR 1) of the N x N level in LDS, in
// place; each wave takes pairs of lines.  SKEW: the level layout above (LP unused); else the
// row pitch LP.
template <int R, int DIR, int NW = kKW, bool SKEW = false>   // NW: waves of the block
__device__ __forceinline__ void dst_lines(double *X, int N, int nl, int LP, const Twiddles<R> &W, double scale,
                                          int wave, int lane) {
  constexpr int M = 64 * R, L = M / 2;
  auto at = [&](int line, int pos) {
    if constexpr (SKEW) return DIR == 0 ? Lvl<R>::at(line, pos) : Lvl<R>::at(pos, line);
    else return DIR == 0 ? line * LP + pos : pos * LP + line;
  };
  const int npairs = (nl + 1) / 2;
  // odd-extension source position and sign of this lane's R values (independent of the pair)
  int srcp[R];
  double sgn[R];
#pragma unroll
  for (int j1 = 0; j1 < R; ++j1) {
    const int jn = 64 * j1 + lane;
    const bool lo = jn >= 1 && jn <= N, hi = jn > L;
    srcp[j1] = lo ? jn - 1 : hi ? M - jn - 1 : 0;
    sgn[j1] = lo ? 1.0 : hi ? -1.0 : 0.0;
  }
  for (int pr = wave; pr < npairs; pr += NW) {
    const int la = 2 * pr, lb = min(2 * pr + 1, nl - 1);
    const double bmask = 2 * pr + 1 < nl ? 1.0 : 0.0;
    double2 v[R];
#pragma unroll
    for (int j1 = 0; j1 < R; ++j1) {
      const double a = X[at(la, srcp[j1])], b = X[at(lb, srcp[j1])];
      v[j1] = make_double2(sgn[j1] * a, sgn[j1] * bmask * b);
    }
    wave_dft<R>(v, lane, W);
    const int k2 = brev6(lane);
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      const int K = k1 + R * k2;
      if (K >= 1 && K <= N) {
        X[at(la, K - 1)] = -v[k1].y * scale;
        if (2 * pr + 1 < nl) X[at(lb, K - 1)] = v[k1].x * scale;
      }
    }
  }
}

// The same for all N lines of an N x N level in the skewed layout.
template <int R, int DIR>
__device__ __forceinline__ void dst_level(double *X, const Twiddles<R> &W, double scale, int wave, int lane) {
  dst_lines<R, DIR, kKW, true>(X, Lvl<R>::N, Lvl<R>::N, 0, W, scale, wave, lane);
}

// X <- U K(a) U X for the level in LDS (U applied as DST along rows, then columns).
template <int R, int KMAX>
__device__ __forceinline__ void uku_level(double *X, const KsP &K, int tid, int wave, int lane) {
  const int N = K.N;
  constexpr int NC = Lvl<R>::N;   // = N (the launcher picks R = (N + 1) / 32): divisions by a constant
  auto at = [](int r, int c) { return Lvl<R>::at(r, c); };
  Twiddles<R> W;
  W.load(reinterpret_cast<const double2 *>(K.tw), lane);
  dst_level<R, 0>(X, W, K.scale, wave, lane);
  __syncthreads();
  dst_level<R, 1>(X, W, K.scale, wave, lane);
  __syncthreads();
  double kv[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int e = tid + k * kKT;
    kv[k] = 0.0;
    if (e < N * N) {
      const int j = e / NC, i = e - j * NC;
      const double uc = X[at(j, i)];
      const double uw = i > 0 ? X[at(j, i - 1)] : 0.0;
      const double ue = i < N - 1 ? X[at(j, i + 1)] : 0.0;
      const double us = j > 0 ? X[at(j - 1, i)] : 0.0;
      const double un = j < N - 1 ? X[at(j + 1, i)] : 0.0;
      const double aw = K.ax[j * (N + 1) + i], ae = K.ax[j * (N + 1) + i + 1];
      const double as = K.ay[j * N + i], an = K.ay[(j + 1) * N + i];
      kv[k] = K.h2inv * (aw * (uc - uw) + ae * (uc - ue) + as * (uc - us) + an * (uc - un));
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int e = tid + k * kKT;
    if (e < N * N) {
      const int j = e / NC, i = e - j * NC;
      X[at(j, i)] = kv[k];
    }
  }
  __syncthreads();
  dst_level<R, 0>(X, W, K.scale, wave, lane);
  __syncthreads();
  dst_level<R, 1>(X, W, K.scale, wave, lane);
  __syncthreads();
}

__device__ __forceinline__ void block_sum4(double (&v)[4], double (*red)[kKW]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s = 0.0;
      for (int w = 0; w < kKW; ++w) s += red[q][w];
      v[q] = s;
    }
}

// MODE 0: q = (T x0)^ (initialising launch).  MODE 1: q = (T z_j)^, the delta partial and,
// when the scalars of launch j-1 cannot exclude convergence, the true residual of the iterate
// that launch j-1 formed.  j = jfull is the index of the fused launch that consumes q.
template <int R, int PR, int MODE>
__device__ __forceinline__ void ks_body(const KsP &K, int jfull, int t) {
  typedef typename std::conditional<PR == 0 || MODE == 0, double, float>::type T;   // source type
  constexpr int KMAX = (R == 4 ? 32 : R == 2 ? 8 : 2);   // ceil(N^2 / 512) for N = 64 R / 2 - 1
  extern __shared__ double X[];
  __shared__ double red[4][kKW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = K.n, m = K.m;
  constexpr int NC = Lvl<R>::N;   // = K.N (the launcher picks R = (N + 1) / 32): divisions by a constant
  auto at = [](int r, int c) { return Lvl<R>::at(r, c); };
  const size_t ld = (size_t)K.ld;
  const int j = jfull % 6;   // rotation phase of the z buffers
  bool do_res = false;
  if (MODE == 1) {
    const Scal *sprev = K.sc + ((j + 1) & 1);   // state after launch j-1
    if (sprev->status != RUNNING) return;
    // the iterate that launch j-1 formed exists from j-1 >= 2 on; its true residual is needed
    // unless sqrt(min sigma) |eta| (a lower bound of ||r||_2, since |eta| = ||r||_{P^-1})
    // still exceeds the tolerance with a margin, or the iteration limit is due
    do_res = jfull >= 3 &&
             (K.sqsigmin * fabs(sprev->eta) <= 2.0 * sprev->rtol * sprev->bnorm || sprev->iter >= sprev->maxit);
  }
  // (T s)^_t = sum_r c_r s_{t-r} + tau U K(a) U (b0 s_t + b1 s_{t-1}): the scheme's time
  // coefficients (theta: 1, -1; BDF-l: alpha_0 .. alpha_l) and weights of K
  double tcs[5], kbs[2];
  const bool far = scheme_coefs(K.scheme, K.theta, tcs, kbs) > 3;   // levels t-3, t-4 enter (BDF3, BDF4)
  const double c0 = tcs[0], c1 = tcs[1], c2 = tcs[2], c3 = tcs[3], c4 = tcs[4];
  const double b0 = kbs[0], b1 = kbs[1];

  double acc_r = 0.0, acc_d = 0.0;
  // ---- q = (T s)^ on level t for the source s (x0 or z_j)
  {
    const T *s = MODE == 0 ? reinterpret_cast<const T *>(K.x)
                           : reinterpret_cast<const T *>(K.Z[(j + 2) % 3]);
    const T *st = s + (size_t)t * ld;
    const T *s1 = t >= 1 ? st - ld : nullptr;
    const T *s2 = t >= 2 ? st - 2 * ld : nullptr;
    const T *s3 = far && t >= 3 ? st - 3 * ld : nullptr;
    const T *s4 = far && t >= 4 ? st - 4 * ld : nullptr;
    for (int e0 = tid; e0 < m; e0 += kLB * kKT) {   // kLB elements' loads in flight
      double a0[kLB], a1[kLB];
#pragma unroll
      for (int u = 0; u < kLB; ++u) {
        const int e = min(e0 + u * kKT, m - 1);
        a0[u] = (double)st[e];
        a1[u] = s1 ? (double)s1[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kLB; ++u) {
        const int e = e0 + u * kKT;
        if (e >= m) break;
        const int jr = e / NC, ir = e - jr * NC;
        X[at(jr, ir)] = b0 * a0[u] + b1 * a1[u];
      }
    }
    __syncthreads();
    uku_level<R, KMAX>(X, K, tid, wave, lane);
    double *q = K.q + (size_t)t * ld;
    const T *sf = s + (size_t)(n - 1 - t) * ld;
    // four elements at a time, all their loads issued before any store of q (a store held
    // back the next element's loads)
    for (int e0 = tid; e0 < m; e0 += 4 * kKT) {
      double a0[4], a1[4], a2[4], af[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * kKT, m - 1);      // past m: a valid element, value unused
        a0[u] = (double)st[e];
        a1[u] = s1 ? (double)s1[e] : 0.0;
        a2[u] = s2 ? (double)s2[e] : 0.0;
        af[u] = MODE == 1 ? (double)sf[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kKT;
        if (e >= m) break;
        const int jr = e / NC, ir = e - jr * NC;
        double v = c0 * a0[u] + c1 * a1[u] + c2 * a2[u] + K.tau * X[at(jr, ir)];
        if (far) v += (s3 ? c3 * (double)s3[e] : 0.0) + (s4 ? c4 * (double)s4[e] : 0.0);
        q[e] = v;
        if (MODE == 1) acc_d += v * af[u];
      }
    }
  }
  // ---- true residual ||b^ - (T x)^||^2 on level t
  if (do_res) {
    __syncthreads();
    const double *xt = K.x + (size_t)t * ld;
    const double *x1 = t >= 1 ? xt - ld : nullptr;
    const double *x2 = t >= 2 ? xt - 2 * ld : nullptr;
    const double *x3 = far && t >= 3 ? xt - 3 * ld : nullptr;
    const double *x4 = far && t >= 4 ? xt - 4 * ld : nullptr;
    const double *bt = K.bh + (size_t)t * ld;
    for (int e0 = tid; e0 < m; e0 += kLB * kKT) {
      double a0[kLB], a1[kLB];
#pragma unroll
      for (int u = 0; u < kLB; ++u) {
        const int e = min(e0 + u * kKT, m - 1);
        a0[u] = xt[e];
        a1[u] = x1 ? x1[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kLB; ++u) {
        const int e = e0 + u * kKT;
        if (e >= m) break;
        const int jr = e / NC, ir = e - jr * NC;
        X[at(jr, ir)] = b0 * a0[u] + b1 * a1[u];
      }
    }
    __syncthreads();
    uku_level<R, KMAX>(X, K, tid, wave, lane);
    for (int e = tid; e < m; e += kKT) {
      const double v0 = xt[e];
      const double v1 = x1 ? x1[e] : 0.0;
      const double v2 = x2 ? x2[e] : 0.0;
      const double v34 = (x3 ? c3 * x3[e] : 0.0) + (x4 ? c4 * x4[e] : 0.0);
      const int jr = e / NC, ir = e - jr * NC;
      const double r = bt[e] - (c0 * v0 + c1 * v1 + c2 * v2 + v34) - K.tau * X[at(jr, ir)];
      acc_r += r * r;
    }
  }
  // ---- partials [residual^2, residual skipped, 0, delta] of this level
  double v[4] = {acc_r, 0.0, 0.0, acc_d};
  block_sum4(v, red);
  if (tid == 0 && MODE == 1) {
    double *pp = K.kpart + 4 * (size_t)t;
    pp[0] = v[0];
    pp[1] = (jfull >= 3 && !do_res) ? 1.0 : 0.0;
    pp[2] = 0.0;
    pp[3] = v[3];
  }
}

// Orthonormal 2D DST-I of every time level in one pass: the level (input slice stride sin)
// goes into LDS, through the row and column transforms, and out with slice stride sout.
// stop_gate: when given, the transform runs only once that scalar state has stopped.
template <int R>
__global__ __launch_bounds__(kKT) void k_dst2d(const double *__restrict__ in, double *__restrict__ out, long sin,
                                               long sout, const double *__restrict__ tw, double scale,
                                               const Scal *__restrict__ stop_gate) {
  if (stop_gate && stop_gate->status == RUNNING) return;
  extern __shared__ double X[];
  constexpr int N = Lvl<R>::N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *src = in + (size_t)blockIdx.x * sin;
  for (int e0 = tid; e0 < N * N; e0 += kLB * kKT) {   // kLB elements' loads in flight
    double a[kLB];
#pragma unroll
    for (int u = 0; u < kLB; ++u) a[u] = src[min(e0 + u * kKT, N * N - 1)];
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = e0 + u * kKT;
      if (e >= N * N) break;
      const int j = e / N, i = e - j * N;
      X[Lvl<R>::at(j, i)] = a[u];
    }
  }
  Twiddles<R> W;
  W.load(reinterpret_cast<const double2 *>(tw), lane);
  __syncthreads();
  dst_level<R, 0>(X, W, scale, wave, lane);
  __syncthreads();
  dst_level<R, 1>(X, W, scale, wave, lane);
  __syncthreads();
  double *dst = out + (size_t)blockIdx.x * sout;
  for (int e = tid; e < N * N; e += kKT) {
    const int j = e / N, i = e - j * N;
    dst[e] = X[Lvl<R>::at(j, i)];
  }
}

template <int R, int PR, int MODE>
__global__ __launch_bounds__(kKT) void k_kslice(KsP K, int jfull) {
  ks_body<R, PR, MODE>(K, jfull, blockIdx.x);
}

// Batched launch: one block per time level of every instance in the table.
template <int R, int PR, int MODE>
__global__ __launch_bounds__(kKT) void k_kslice_multi(const KsP *__restrict__ table, int ninst, int jfull) {
  const int b = blockIdx.x;
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const KsP &K = table[lo];   // read in place (a private copy would go to scratch)
  ks_body<R, PR, MODE>(K, jfull, b - K.blk0);
}

template <int R, int PR>
size_t ks_shmem() { return (size_t)Lvl<R>::SIZE * sizeof(double); }

template <int R, int PR>
hipError_t run_ks(hipStream_t st, const KsP *K, const KsP *table, int ninst, int blocks, int mode, int jfull) {
  const size_t sh = ks_shmem<R, PR>();
  if (sh > 65536) {
    lds_limit((const void *)k_kslice<R, PR, 0>, sh);
    lds_limit((const void *)k_kslice<R, PR, 1>, sh);
    lds_limit((const void *)k_kslice_multi<R, PR, 0>, sh);
    lds_limit((const void *)k_kslice_multi<R, PR, 1>, sh);
  }
  if (K) {
    if (mode == 0) hipLaunchKernelGGL((k_kslice<R, PR, 0>), dim3(blocks), dim3(kKT), sh, st, *K, jfull);
    else hipLaunchKernelGGL((k_kslice<R, PR, 1>), dim3(blocks), dim3(kKT), sh, st, *K, jfull);
  } else {
    if (mode == 0) hipLaunchKernelGGL((k_kslice_multi<R, PR, 0>), dim3(blocks), dim3(kKT), sh, st, table, ninst, jfull);
    else hipLaunchKernelGGL((k_kslice_multi<R, PR, 1>), dim3(blocks), dim3(kKT), sh, st, table, ninst, jfull);
  }
  return hipGetLastError();
}

template <int PR>
hipError_t run_ks_r(hipStream_t st, int L, const KsP *K, const KsP *table, int ninst, int blocks, int mode, int jfull) {
  switch (L) {
    case 32: return run_ks<1, PR>(st, K, table, ninst, blocks, mode, jfull);
    case 64: return run_ks<2, PR>(st, K, table, ninst, blocks, mode, jfull);
    case 128: return run_ks<4, PR>(st, K, table, ninst, blocks, mode, jfull);
    default: break;
  }
  return hipErrorInvalidValue;
}

// ---- The per-level matvec at N = 127 as three streamed passes over line tiles.
// U K(a) U s per level, with U = S_y S_x: (A) row transforms of the source, s = b0 z_t +
// b1 z_{t-1}, into Y1; (B) per tile of 16 columns: the column transforms of those columns and
// of one halo column on each side, the 5-point stencil K(a) on the 16, and their column
// transforms back, into Y2; (C) row transforms of Y2, combined with the time stencil into
// q_t = sum_r c_r z_{t-r} + tau (U K U s)_t, with the delta partial per tile.  A block holds
// at most 18 lines (18.6 KB of LDS) instead of a whole level (139 KB), so several blocks
// share a CU and one block's loads overlap another's transforms.  The true-residual chain
// runs the same three passes on x in the same launches, through intermediates of its own,
// when launch j-1's scalars ask for it.  Same arithmetic as the level kernel; only the
// partial sums are grouped per tile (kKsTiles per level).
constexpr int kKsN = 127, kKsLP = kKsN + 2;   // level size, LDS pitch of a line
constexpr int kKsTT = 256;                     // threads per block: 4 waves
constexpr int kKsTL = 16;                      // rows (passes A, C) or columns (pass B) per tile
static_assert(kKsTiles * kKsTL >= kKsN && (kKsTiles - 1) * kKsTL < kKsN, "tiles cover a level");


__device__ __forceinline__ double block_sum_tt(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kKsTT / 64; ++w) s += red[w];
  return s;
}

// Pass A: Y1_t = S_x (b0 s_t + b1 s_{t-1}) on rows [16 tile, 16 tile + 16) of level t; s = x
// (MODE 0, residual chain) or z_j.
template <int PR, int MODE, bool RES>
__device__ __forceinline__ void ks_rows_in(const KsP &K, int jfull, int t, int tile, double *X, double *yout) {
  typedef typename std::conditional<PR == 0 || MODE == 0 || RES, double, float>::type T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = tile * kKsTL, nl = min(kKsTL, kKsN - r0);
  const size_t ld = (size_t)K.ld;
  double tcs[5], kbs[2];
  (void)scheme_coefs(K.scheme, K.theta, tcs, kbs);
  const double b0 = kbs[0], b1 = kbs[1];
  const T *s = MODE == 0 || RES ? reinterpret_cast<const T *>(K.x)
                                : reinterpret_cast<const T *>(K.Z[((jfull % 6) + 2) % 3]);
  const T *st = s + (size_t)t * ld + (size_t)r0 * kKsN;      // the tile's rows are contiguous
  const T *s1 = t >= 1 ? st - ld : nullptr;
  for (int e0 = tid; e0 < nl * kKsN; e0 += kLB * kKsTT) {
    double a0[kLB], a1[kLB];
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = min(e0 + u * kKsTT, nl * kKsN - 1);
      a0[u] = (double)st[e];
      a1[u] = s1 ? (double)s1[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = e0 + u * kKsTT;
      if (e >= nl * kKsN) break;
      const int c = e / kKsN, i = e - c * kKsN;
      X[c * kKsLP + i] = b0 * a0[u] + b1 * a1[u];
    }
  }
  Twiddles<4> W;
  W.load(reinterpret_cast<const double2 *>(K.tw), lane);
  __syncthreads();
  dst_lines<4, 0, kKsTT / 64>(X, kKsN, nl, kKsLP, W, K.scale, wave, lane);
  __syncthreads();
  double *y = yout + (size_t)t * ld + (size_t)r0 * kKsN;
  for (int e = tid; e < nl * kKsN; e += kKsTT) {
    const int c = e / kKsN, i = e - c * kKsN;
    y[e] = X[c * kKsLP + i];
  }
}

// Pass B: columns [16 tile, 16 tile + 16) of Y2_t = S_y K(a) S_y Y1_t (the halo columns
// c0 - 1 and c1 are transformed as well, for the stencil's x neighbours).
// X: (kKsTL + 2) lines of kKsLP (line = column, position = row).
__device__ __forceinline__ void ks_cols(const KsP &K, int t, int tile, double *X, const double *yin, double *yout) {
  constexpr int N = kKsN, LP = kKsLP;
  constexpr int KV = (kKsTL * kKsN + kKsTT - 1) / kKsTT;   // stencil points per thread
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = tile * kKsTL, c1 = min(N, c0 + kKsTL), nin = c1 - c0;
  const int cl = max(0, c0 - 1), ch = min(N, c1 + 1), nh = ch - cl;
  const size_t ld = (size_t)K.ld;
  const double *y1 = yin + (size_t)t * ld;
  for (int e0 = tid; e0 < N * nh; e0 += kLB * kKsTT) {
    double a[kLB];
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = min(e0 + u * kKsTT, N * nh - 1);
      const int r = e / nh, c = e - r * nh;
      a[u] = y1[(size_t)r * N + cl + c];
    }
#pragma unroll
    for (int u = 0; u < kLB; ++u) {
      const int e = e0 + u * kKsTT;
      if (e >= N * nh) break;
      const int r = e / nh, c = e - r * nh;
      X[c * LP + r] = a[u];
    }
  }
  Twiddles<4> W;
  W.load(reinterpret_cast<const double2 *>(K.tw), lane);
  __syncthreads();
  dst_lines<4, 0, kKsTT / 64>(X, N, nh, LP, W, K.scale, wave, lane);
  __syncthreads();
  // K(a) u on the tile's columns: u(r, c) = X[(c - cl) LP + r], zero beyond the boundary
  double kv[KV];
#pragma unroll
  for (int k = 0; k < KV; ++k) {
    const int e = tid + k * kKsTT;
    kv[k] = 0.0;
    if (e < nin * N) {
      const int r = e / nin, c = c0 + (e - r * nin);
      const double *xc = X + (c - cl) * LP;
      const double uc = xc[r];
      const double uw = c > 0 ? xc[r - LP] : 0.0;
      const double ue = c < N - 1 ? xc[r + LP] : 0.0;
      const double us = r > 0 ? xc[r - 1] : 0.0;
      const double un = r < N - 1 ? xc[r + 1] : 0.0;
      const double aw = K.ax[r * (N + 1) + c], ae = K.ax[r * (N + 1) + c + 1];
      const double as = K.ay[r * N + c], an = K.ay[(r + 1) * N + c];
      kv[k] = K.h2inv * (aw * (uc - uw) + ae * (uc - ue) + as * (uc - us) + an * (uc - un));
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KV; ++k) {
    const int e = tid + k * kKsTT;
    if (e < nin * N) {
      const int r = e / nin, c = e - r * nin;
      X[c * LP + r] = kv[k];
    }
  }
  __syncthreads();
  dst_lines<4, 0, kKsTT / 64>(X, N, nin, LP, W, K.scale, wave, lane);
  __syncthreads();
  double *y2 = yout + (size_t)t * ld;
  for (int e = tid; e < nin * N; e += kKsTT) {
    const int r = e / nin, c = e - r * nin;
    y2[(size_t)r * N + c0 + c] = X[c * LP + r];
  }
}

// Pass C: rows [16 tile, 16 tile + 16) of S_x Y2_t, then q_t = sum_r c_r s_{t-r} + tau (.)
// with the delta partial of the tile (source chain), or the tile's part of
// ||b^ - (T x)^||^2 (residual chain).  Partials: 4 per (level, tile), [residual^2, residual
// skipped, 0, delta]; the residual chain runs after the source chain and fills slot 0.
template <int PR, int MODE, bool RES>
__device__ __forceinline__ void ks_rows_out(const KsP &K, int jfull, int t, int tile, bool skipped, double *X,
                                            double *red, const double *yin) {
  typedef typename std::conditional<PR == 0 || MODE == 0 || RES, double, float>::type T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = tile * kKsTL, nl = min(kKsTL, kKsN - r0), ne = nl * kKsN;
  const int n = K.n;
  const size_t ld = (size_t)K.ld, o = (size_t)r0 * kKsN;
  const double *y2 = yin + (size_t)t * ld + o;
  for (int e = tid; e < ne; e += kKsTT) {
    const int c = e / kKsN, i = e - c * kKsN;
    X[c * kKsLP + i] = y2[e];
  }
  Twiddles<4> W;
  W.load(reinterpret_cast<const double2 *>(K.tw), lane);
  __syncthreads();
  dst_lines<4, 0, kKsTT / 64>(X, kKsN, nl, kKsLP, W, K.scale, wave, lane);
  __syncthreads();
  double tcs[5], kbs[2];
  const bool far = scheme_coefs(K.scheme, K.theta, tcs, kbs) > 3;   // levels t-3, t-4 enter (BDF3, BDF4)
  const double c0 = tcs[0], c1 = tcs[1], c2 = tcs[2], c3 = tcs[3], c4 = tcs[4];
  const T *s = MODE == 0 || RES ? reinterpret_cast<const T *>(K.x)
                                : reinterpret_cast<const T *>(K.Z[((jfull % 6) + 2) % 3]);
  const T *st = s + (size_t)t * ld + o;
  const T *s1 = t >= 1 ? st - ld : nullptr;
  const T *s2 = t >= 2 ? st - 2 * ld : nullptr;
  const T *s3 = far && t >= 3 ? st - 3 * ld : nullptr;
  const T *s4 = far && t >= 4 ? st - 4 * ld : nullptr;
  double acc = 0.0;
  if (!RES) {
    double *q = K.q + (size_t)t * ld + o;
    const T *sf = s + (size_t)(n - 1 - t) * ld + o;
    for (int e0 = tid; e0 < ne; e0 += 4 * kKsTT) {   // four elements' loads in flight
      double a0[4], a1[4], a2[4], af[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * kKsTT, ne - 1);
        a0[u] = (double)st[e];
        a1[u] = s1 ? (double)s1[e] : 0.0;
        a2[u] = s2 ? (double)s2[e] : 0.0;
        af[u] = MODE == 1 ? (double)sf[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kKsTT;
        if (e >= ne) break;
        const int c = e / kKsN, i = e - c * kKsN;
        double v = c0 * a0[u] + c1 * a1[u] + c2 * a2[u] + K.tau * X[c * kKsLP + i];
        if (far) v += (s3 ? c3 * (double)s3[e] : 0.0) + (s4 ? c4 * (double)s4[e] : 0.0);
        q[e] = v;
        if (MODE == 1) acc += v * af[u];
      }
    }
  } else {
    const double *bt = K.bh + (size_t)t * ld + o;
    for (int e0 = tid; e0 < ne; e0 += 4 * kKsTT) {
      double v0[4], v1[4], v2[4], v34[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * kKsTT, ne - 1);
        v0[u] = (double)st[e];
        v1[u] = s1 ? (double)s1[e] : 0.0;
        v2[u] = s2 ? (double)s2[e] : 0.0;
        v34[u] = (s3 ? c3 * (double)s3[e] : 0.0) + (s4 ? c4 * (double)s4[e] : 0.0);
        bb[u] = bt[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kKsTT;
        if (e >= ne) break;
        const int c = e / kKsN, i = e - c * kKsN;
        const double r = bb[u] - (c0 * v0[u] + c1 * v1[u] + c2 * v2[u] + v34[u]) - K.tau * X[c * kKsLP + i];
        acc += r * r;
      }
    }
  }
  if (MODE == 0) return;
  const double sum = block_sum_tt(acc, red);
  if (tid == 0) {
    double *pp = K.kpart + 4 * ((size_t)t * kKsTiles + tile);
    if (RES) {
      pp[0] = sum;
    } else {
      pp[0] = 0.0;
      pp[1] = skipped ? 1.0 : 0.0;
      pp[2] = 0.0;
      pp[3] = sum;
    }
  }
}

// One pass on one tile: the source chain, then (MODE 1) the residual chain on x when the
// scalars of launch j - 1 cannot exclude convergence (the level kernel's rule); MODE 0
// (q = (T x0)^) has no residual.  Nothing runs once the solve has stopped.
template <int PASS, int PR, int MODE>
__device__ __forceinline__ void ks_pass(const KsP &K, int jfull, int t, int tile) {
  __shared__ double X[(kKsTL + 2) * kKsLP];
  __shared__ double red[kKsTT / 64];
  bool do_res = false, skipped = false;
  if (MODE == 1) {
    const Scal *sprev = K.sc + (((jfull % 6) + 1) & 1);
    if (sprev->status != RUNNING) return;
    do_res = jfull >= 3 &&
             (K.sqsigmin * fabs(sprev->eta) <= 2.0 * sprev->rtol * sprev->bnorm || sprev->iter >= sprev->maxit);
    skipped = jfull >= 3 && !do_res;
  }
  // the source chain passes its intermediates through y[0], y[1], the residual chain through
  // y[2], y[3] (both run in the same launches)
  if (PASS == 0) ks_rows_in<PR, MODE, false>(K, jfull, t, tile, X, K.y[0]);
  else if (PASS == 1) ks_cols(K, t, tile, X, K.y[0], K.y[1]);
  else ks_rows_out<PR, MODE, false>(K, jfull, t, tile, skipped, X, red, K.y[1]);
  if (MODE == 1 && do_res) {
    __syncthreads();
    if (PASS == 0) ks_rows_in<PR, MODE, true>(K, jfull, t, tile, X, K.y[2]);
    else if (PASS == 1) ks_cols(K, t, tile, X, K.y[2], K.y[3]);
    else ks_rows_out<PR, MODE, true>(K, jfull, t, tile, skipped, X, red, K.y[3]);
  }
}
// Single plan: block (t, tile); batched: the table's instances, level blocks counted by blk0.
template <int PASS, int PR, int MODE>
__global__ __launch_bounds__(kKsTT) void k_ks_tiles(KsP K, int jfull) {
  const int b = xcd_block(blockIdx.x, gridDim.x), t = b / kKsTiles;
  ks_pass<PASS, PR, MODE>(K, jfull, t, b - t * kKsTiles);
}
template <int PASS, int PR, int MODE>
__global__ __launch_bounds__(kKsTT) void k_ks_tiles_multi(const KsP *__restrict__ table, int ninst, int jfull) {
  const int b = xcd_block(blockIdx.x, gridDim.x), g = b / kKsTiles;
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].blk0 <= g) lo = mid;
    else hi = mid - 1;
  }
  const KsP &K = table[lo];
  ks_pass<PASS, PR, MODE>(K, jfull, g - K.blk0, b - g * kKsTiles);
}

// The chain of one launch: passes A, B, C of the source, then (MODE 1) of the residual, whose
// blocks exit at once unless launch j-1's scalars ask for it.  levels: grid / kKsTiles.
// The three passes of one launch (levels: grid / kKsTiles).
template <int PR, int MODE>
hipError_t run_ks_chain(hipStream_t st, const KsP *K, const KsP *table, int ninst, int levels, int jfull) {
  const dim3 g(levels * kKsTiles), blk(kKsTT);
  if (K) {
    hipLaunchKernelGGL((k_ks_tiles<0, PR, MODE>), g, blk, 0, st, *K, jfull);
    hipLaunchKernelGGL((k_ks_tiles<1, PR, MODE>), g, blk, 0, st, *K, jfull);
    hipLaunchKernelGGL((k_ks_tiles<2, PR, MODE>), g, blk, 0, st, *K, jfull);
  } else {
    hipLaunchKernelGGL((k_ks_tiles_multi<0, PR, MODE>), g, blk, 0, st, table, ninst, jfull);
    hipLaunchKernelGGL((k_ks_tiles_multi<1, PR, MODE>), g, blk, 0, st, table, ninst, jfull);
    hipLaunchKernelGGL((k_ks_tiles_multi<2, PR, MODE>), g, blk, 0, st, table, ninst, jfull);
  }
  return hipGetLastError();
}
template <int PR>
hipError_t run_ks_split(hipStream_t st, const KsP *K, const KsP *table, int ninst, int levels, int mode, int jfull) {
  return mode == 0 ? run_ks_chain<PR, 0>(st, K, table, ninst, levels, jfull)
                   : run_ks_chain<PR, 1>(st, K, table, ninst, levels, jfull);
}

}  // namespace

namespace {

// One spatial DST-I pass over a 2D field (N + 1 = 32 R): along x (DIR 0, rows) or y (DIR 1,
// columns) of every time slice.  A block owns up to kTL lines of one slice, loads them
// coalesced into LDS (rows: contiguous; columns: kTL neighbours per row), every wave takes a
// line pair through the register FFT, and the block stores them back (all loads finish before
// any store, so in == out is allowed).  Small tiles keep many blocks per CU, so that some
// stream while others transform.  N + 1 = 256 runs the persistent variant further down.
// scale_mode 1 divides by the Chebyshev inner diagonal ez[s] + ez[n + s] abar tmu_lap[q].
constexpr int kTL = 8;
constexpr int kTT = 256;    // threads of a tile block: one line pair per wave
struct TileP {
  int N, n, tiles;            // tiles per slice
  long sin, sout;
  double scale, abar;
  const double *tw, *ez, *tmu_lap;
  int scale_mode;
  // scale_mode 3 (row passes, N + 1 = 256): the Chebyshev update takes the result t instead
  // of a store: dv = a_t t (cfirst) or a_d dv + a_t t, then x = dv (cfirst) or x + dv
  void *cx, *cd;
  double ca_d, ca_t;
  int cfirst;
};

// TI, TO: element types of the vectors in memory (float32 intermediates of a mixed-precision
// P^{-1}); the tile in LDS and the FFT stay float64.
// TL: lines per tile (8, or 16 in column passes when tuned: a tile's row piece is then 128
// bytes of float64 or 64 of float32).
template <int R, int DIR, typename TI, typename TO, int TL>
__global__ __launch_bounds__(kTT) void k_dst_tile(TileP d, const TI *__restrict__ in, TO *__restrict__ out,
                                                  const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  extern __shared__ double X[];
  constexpr int N = 32 * R - 1;
  constexpr int LP = DIR == 0 ? N + 2 : TL + 1;    // LDS pitch of a line (DIR 0) or a position (DIR 1)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int s = bid / d.tiles, i0 = (bid - s * d.tiles) * TL;
  const int nl = min(TL, N - i0);
  const TI *src = in + (size_t)s * d.sin;
  TO *dst = out + (size_t)s * d.sout;
  Twiddles<R> W;
  W.load(reinterpret_cast<const double2 *>(d.tw), lane);
  if (DIR == 0) {
    for (int e = tid; e < nl * N; e += kTT) {           // rows i0.. are contiguous
      const int c = e / N, j = e - c * N;
      X[c * LP + j] = (double)src[(size_t)i0 * N + e];
    }
  } else {
    for (int e = tid; e < TL * N; e += kTT) {
      const int j = e / TL, c = e - j * TL;
      if (c < nl) X[j * LP + c] = (double)src[(size_t)j * N + i0 + c];
    }
  }
  __syncthreads();
  dst_lines<R, DIR, kTT / 64>(X, N, nl, LP, W, d.scale, wave, lane);
  __syncthreads();
  auto fin = [&](double v, size_t q) {
    return d.scale_mode == 1 ? v / (d.ez[s] + d.ez[d.n + s] * d.abar * d.tmu_lap[q]) : v;
  };
  if (DIR == 0) {
    for (int e = tid; e < nl * N; e += kTT) {
      const int c = e / N, j = e - c * N;
      const size_t q = (size_t)i0 * N + e;
      dst[q] = (TO)fin(X[c * LP + j], q);
    }
  } else {
    for (int e = tid; e < TL * N; e += kTT) {
      const int j = e / TL, c = e - j * TL;
      if (c < nl) {
        const size_t q = (size_t)j * N + i0 + c;
        dst[q] = (TO)fin(X[j * LP + c], q);
      }
    }
  }
}

// N + 1 = 256 (M = 512): the line pair's DFT regroups its values through LDS instead of six
// cross-lane exchange stages.  With n = 64 n1 + n2 (n2 = lane) and k = k1 + 8 k2, an in-lane
// 8-point DFT over n1 and the twiddle W_512^{n2 k1} leave a 64-point DFT over n2 for every k1;
// it is split as n2 = 8 a + b, k2 = c + 8 d into an 8-point DFT over a, the twiddle
// W_64^{b c} and an 8-point DFT over b, each done in-lane after the values are regrouped in
// LDS (real parts, then imaginary parts).  On return lane 8 k1 + c holds Z[k1 + 8 c + 64 d]
// in v[d].  T: this wave's 8 rows of kTP doubles; every wave of the block must call it.
constexpr int kTP = 72;    // row pitch of the regrouping buffer (64 values + one pad per 8)
__device__ __forceinline__ void pair_dft512(double2 (&v)[8], int lane, const double2 (&wa)[7],
                                            const double2 (&wb)[7], double *T) {
  lane_dft8(v);                                                   // over n1 -> k1
#pragma unroll
  for (int k1 = 1; k1 < 8; ++k1) v[k1] = cmul(v[k1], wa[k1 - 1]);   // W_512^{n2 k1}
  const int rk = lane >> 3, rb = lane & 7;                          // reader: k1, b
#pragma unroll
  for (int part = 0; part < 2; ++part) {     // lane n2 writes row k1 at n2 + n2 / 8
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) T[k1 * kTP + lane + (lane >> 3)] = part == 0 ? v[k1].x : v[k1].y;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double t = T[rk * kTP + 9 * a + rb];                  // n2 = 8 a + b
      if (part == 0) v[a].x = t; else v[a].y = t;
    }
    __syncthreads();
  }
  lane_dft8(v);                                                   // over a -> c
#pragma unroll
  for (int c = 1; c < 8; ++c) v[c] = cmul(v[c], wb[c - 1]);        // W_64^{b c}
#pragma unroll
  for (int part = 0; part < 2; ++part) {     // lane (k1, b) writes row k1 at 9 c + b
#pragma unroll
    for (int c = 0; c < 8; ++c) T[rk * kTP + 9 * c + rb] = part == 0 ? v[c].x : v[c].y;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 8; ++b) {                                 // reader: k1, c = lane % 8
      const double t = T[rk * kTP + 9 * rb + b];
      if (part == 0) v[b].x = t; else v[b].y = t;
    }
    __syncthreads();
  }
  lane_dft8(v);                                                   // over b -> d
}

// One DST-I pass for N + 1 = 256.  Persistent blocks walk the tiles of an XCD-contiguous
// range, holding the next tile's loads in registers while the current tile is transformed
// (loads of one tile and stores of another touch different lines, so in == out is allowed);
// the regrouping buffers alias the tile once the line pairs are in registers.
// NWV waves, one line pair each: tiles of 2 NWV lines (8 lines, or 16 in column passes when
// tuned, for longer row pieces).  scale_mode 1 divides the result by the Chebyshev inner
// diagonal on the way out; scale_mode 2 (column passes) divides it in the tile and takes the
// tile through the same transform again: the two consecutive column passes of the inner
// preconditioner in one read and one write of the vector.
template <int DIR, typename TI, typename TO, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_dst_tile512(TileP d, const TI *__restrict__ in,
                                                          TO *__restrict__ out, const Scal *__restrict__ gate,
                                                          int total) {
  if (gate && gate->status != RUNNING) return;
  constexpr int kTT = 64 * NWV;
  constexpr int kLds512 = NWV * 8 * kTP;   // doubles: >= one tile in either direction
  __shared__ double X[kLds512];
  constexpr int N = 255, M = 512, L = 256, TL = 2 * NWV, TILES = (N + TL - 1) / TL;
  constexpr int LP = DIR == 0 ? N + 2 : TL + 1;
  constexpr int PF = (TL * N + kTT - 1) / kTT;
  static_assert((DIR == 0 ? TL * LP : N * LP) <= kLds512, "the tile fits");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *T = X + wave * 8 * kTP;
  const int xcd = blockIdx.x % 8, nbx = gridDim.x / 8;
  const int per = (total + 7) / 8, tend = min(total, (xcd + 1) * per);
  const double2 *tw = reinterpret_cast<const double2 *>(d.tw);
  double2 wa[7], wb[7];
#pragma unroll
  for (int k = 1; k < 8; ++k) {
    wa[k - 1] = twid(tw, lane * k, M);
    wb[k - 1] = twid(tw, 8 * (lane & 7) * k, M);
  }
  auto at = [&](int line, int pos) { return DIR == 0 ? line * LP + pos : pos * LP + line; };
  double pre[PF];
  auto load = [&](int t) {
    const int s = t / TILES, i0 = (t - s * TILES) * TL, nl = min(TL, N - i0);
    const TI *src = in + (size_t)s * d.sin;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * kTT;
      if (DIR == 0) {
        pre[k] = e < nl * N ? (double)src[(size_t)i0 * N + e] : 0.0;       // rows i0.. are contiguous
      } else {
        const int j = e / TL, c = e - j * TL;
        pre[k] = (e < TL * N && c < nl) ? (double)src[(size_t)j * N + i0 + c] : 0.0;
      }
    }
  };
  int t = xcd * per + blockIdx.x / 8;
  if (t < tend) load(t);
  for (; t < tend; t += nbx) {
    const int s = t / TILES, i0 = (t - s * TILES) * TL, nl = min(TL, N - i0);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * kTT;
      if (DIR == 0) {
        if (e < nl * N) {
          const int c = e / N, j = e - c * N;
          X[c * LP + j] = pre[k];
        }
      } else if (e < TL * N) {
        const int j = e / TL, c = e - j * TL;
        X[j * LP + c] = pre[k];
      }
    }
    __syncthreads();
    if (t + nbx < tend) load(t + nbx);
    // the wave's line pair, oddly extended to M points (lines past nl read as zero)
    const int la = min(2 * wave, nl - 1), lb = min(2 * wave + 1, nl - 1);
    const bool oka = 2 * wave < nl, okb = 2 * wave + 1 < nl;
    // the tile's lines through the DST, results back in the tile
    auto transform = [&]() {
      double2 v[8];
#pragma unroll
      for (int j1 = 0; j1 < 8; ++j1) {
        const int jn = 64 * j1 + lane;
        const bool lo = jn >= 1 && jn <= N, hi = jn > L;
        const int sp = lo ? jn - 1 : hi ? M - jn - 1 : 0;
        const double sg = lo ? 1.0 : hi ? -1.0 : 0.0;
        v[j1] = make_double2(oka ? sg * X[at(la, sp)] : 0.0, okb ? sg * X[at(lb, sp)] : 0.0);
      }
      __syncthreads();
      pair_dft512(v, lane, wa, wb, T);
      __syncthreads();
      // (S a)_k = -Im Z_{k+1} / sqrt(2L), (S b)_k = Re Z_{k+1} / sqrt(2L); k + 1 < 256 needs d < 4
      const int k1 = lane >> 3, c = lane & 7;
#pragma unroll
      for (int dd = 0; dd < 4; ++dd) {
        const int K = k1 + 8 * c + 64 * dd;
        if (K >= 1) {
          if (oka) X[at(la, K - 1)] = -v[dd].y * d.scale;
          if (okb) X[at(lb, K - 1)] = v[dd].x * d.scale;
        }
      }
      __syncthreads();
    };
    transform();
    if (DIR == 1 && d.scale_mode == 2) {
      // the diagonal division between two column passes, in the tile, then the second pass
      for (int e = tid; e < TL * N; e += kTT) {
        const int j = e / TL, c2 = e - j * TL;
        if (c2 < nl) {
          const size_t q = (size_t)j * N + i0 + c2;
          X[j * LP + c2] /= d.ez[s] + d.ez[d.n + s] * d.abar * d.tmu_lap[q];
        }
      }
      __syncthreads();
      transform();
    }
    TO *dst = out + (size_t)s * d.sout;
    auto fin = [&](double x, size_t q) {
      return d.scale_mode == 1 ? x / (d.ez[s] + d.ez[d.n + s] * d.abar * d.tmu_lap[q]) : x;
    };
    if (DIR == 0 && d.scale_mode == 3) {
      TO *xv = reinterpret_cast<TO *>(d.cx) + (size_t)s * d.sout;
      TO *dv = reinterpret_cast<TO *>(d.cd) + (size_t)s * d.sout;
      for (int e = tid; e < nl * N; e += kTT) {
        const int c2 = e / N, j = e - c2 * N;
        const size_t q = (size_t)i0 * N + e;
        const double tv = (double)(TO)X[c2 * LP + j];     // the result as a stored vector holds it
        const double dn = d.cfirst ? d.ca_t * tv : d.ca_d * (double)dv[q] + d.ca_t * tv;
        dv[q] = (TO)dn;
        xv[q] = d.cfirst ? (TO)dn : (TO)((double)xv[q] + dn);
      }
    } else if (DIR == 0) {
      for (int e = tid; e < nl * N; e += kTT) {
        const int c2 = e / N, j = e - c2 * N;
        const size_t q = (size_t)i0 * N + e;
        dst[q] = (TO)fin(X[c2 * LP + j], q);
      }
    } else {
      for (int e = tid; e < TL * N; e += kTT) {
        const int j = e / TL, c2 = e - j * TL;
        if (c2 < nl) {
          const size_t q = (size_t)j * N + i0 + c2;
          dst[q] = (TO)fin(X[j * LP + c2], q);
        }
      }
    }
    __syncthreads();
  }
}

// resident blocks of the persistent pass (LDS allows 8 four-wave blocks per CU); measured at
// N = 255, n = 512; eight-wave blocks: half as many
constexpr int kGrid512[2] = {2048, 4096};

template <int R, typename TI, typename TO>
hipError_t run_dst_tile(hipStream_t st, int dir, TileP d, int nslices, const TI *in, TO *out, const Scal *gate,
                        bool col16) {
  const int TLr = (dir == 1 && col16) ? 16 : kTL;   // lines per tile of this pass
  d.tiles = (d.N + TLr - 1) / TLr;
  if constexpr (R == 8) {
    const long total = (long)nslices * d.tiles;
    if (TLr == 16) {
      const int grid = (int)std::min<long>(kGrid512[dir] / 2, (total + 7) / 8 * 8);
      hipLaunchKernelGGL((k_dst_tile512<1, TI, TO, 8>), dim3(grid), dim3(512), 0, st, d, in, out, gate, (int)total);
    } else {
      const int grid = (int)std::min<long>(kGrid512[dir], (total + 7) / 8 * 8);
      if (dir == 0)
        hipLaunchKernelGGL((k_dst_tile512<0, TI, TO, 4>), dim3(grid), dim3(kTT), 0, st, d, in, out, gate, (int)total);
      else
        hipLaunchKernelGGL((k_dst_tile512<1, TI, TO, 4>), dim3(grid), dim3(kTT), 0, st, d, in, out, gate, (int)total);
    }
  } else {
    constexpr int N = 32 * R - 1;
    const size_t sh = (size_t)(dir == 0 ? TLr * (N + 2) : N * (TLr + 1)) * sizeof(double);
    const void *f = dir == 0 ? (const void *)k_dst_tile<R, 0, TI, TO, kTL>
                             : TLr == 16 ? (const void *)k_dst_tile<R, 1, TI, TO, 16>
                                         : (const void *)k_dst_tile<R, 1, TI, TO, kTL>;
    if (sh > 65536) {
      const hipError_t e = lds_limit(f, sh);
      if (e != hipSuccess) return e;
    }
    const unsigned blocks = (unsigned)((long)nslices * d.tiles);
    if (dir == 0)
      hipLaunchKernelGGL((k_dst_tile<R, 0, TI, TO, kTL>), dim3(blocks), dim3(kTT), sh, st, d, in, out, gate);
    else if (TLr == 16)
      hipLaunchKernelGGL((k_dst_tile<R, 1, TI, TO, 16>), dim3(blocks), dim3(kTT), sh, st, d, in, out, gate);
    else
      hipLaunchKernelGGL((k_dst_tile<R, 1, TI, TO, kTL>), dim3(blocks), dim3(kTT), sh, st, d, in, out, gate);
  }
  return hipGetLastError();
}

}  // namespace

bool dst_tile_supported(const Plan *p) {
  return p->dim == 2 && (p->L == 32 || p->L == 64 || p->L == 128 || p->L == 256);
}

namespace {
template <int R>
hipError_t run_dst_tile_v(hipStream_t st, int dir, const TileP &d, int nslices, const void *in, bool in32, void *out,
                          bool out32, const Scal *gate, bool col16) {
  if (!in32 && !out32) return run_dst_tile<R>(st, dir, d, nslices, (const double *)in, (double *)out, gate, col16);
  if (!in32 && out32) return run_dst_tile<R>(st, dir, d, nslices, (const double *)in, (float *)out, gate, col16);
  if (in32 && out32) return run_dst_tile<R>(st, dir, d, nslices, (const float *)in, (float *)out, gate, col16);
  return run_dst_tile<R>(st, dir, d, nslices, (const float *)in, (double *)out, gate, col16);
}
}  // namespace

hipError_t launch_dst_tile(Ctx c, int dir, const void *in, bool in32, void *out, bool out32, int nslices,
                           int scale_mode, const Scal *gate, long in_stride, long out_stride, bool col16) {
  const Plan *p = c.p;
  if (!dst_tile_supported(p) || dir < 0 || dir > 1) return hipErrorInvalidValue;
  TileP d{};
  d.N = p->N;
  d.n = p->n;
  d.tiles = (p->N + kTL - 1) / kTL;
  d.sin = in_stride ? in_stride : p->m;
  d.sout = out_stride ? out_stride : p->m;
  d.scale = 1.0 / sqrt(2.0 * p->L);
  d.abar = p->abar;
  d.tw = p->tw;
  d.ez = p->ez;
  d.tmu_lap = p->tmu_lap;
  d.scale_mode = scale_mode;
  // scale_mode 2 (divide, then the same column pass again) exists for N + 1 = 256 only, and
  // scale_mode 3 (the Chebyshev update) only through launch_dst_cheb_axpy
  if ((scale_mode == 2 && (p->L != 256 || dir != 1)) || scale_mode == 3) return hipErrorInvalidValue;
  switch (p->L) {
    case 32: return run_dst_tile_v<1>(c.st, dir, d, nslices, in, in32, out, out32, gate, col16);
    case 64: return run_dst_tile_v<2>(c.st, dir, d, nslices, in, in32, out, out32, gate, col16);
    case 128: return run_dst_tile_v<4>(c.st, dir, d, nslices, in, in32, out, out32, gate, col16);
    case 256: return run_dst_tile_v<8>(c.st, dir, d, nslices, in, in32, out, out32, gate, col16);
    default: break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dst_cheb_axpy(Ctx c, const void *in, void *x, void *dvec, bool f32, double a_d, double a_t,
                                int first, const Scal *gate) {
  const Plan *p = c.p;
  if (!dst_tile_supported(p) || p->L != 256) return hipErrorInvalidValue;
  TileP d{};
  d.N = p->N;
  d.n = p->n;
  d.tiles = (p->N + kTL - 1) / kTL;
  d.sin = d.sout = p->m;
  d.scale = 1.0 / sqrt(2.0 * p->L);
  d.abar = p->abar;
  d.tw = p->tw;
  d.ez = p->ez;
  d.tmu_lap = p->tmu_lap;
  d.scale_mode = 3;
  d.cx = x;
  d.cd = dvec;
  d.ca_d = a_d;
  d.ca_t = a_t;
  d.cfirst = first;
  return run_dst_tile_v<8>(c.st, 0, d, p->n, in, f32, x, f32, gate, false);
}

bool kslice_supported(const Plan *p) { return p->dim == 2 && (p->L == 32 || p->L == 64 || p->L == 128); }

template <int R>
static hipError_t run_dst2d(hipStream_t st, int n, const double *in, double *out, long sin, long sout,
                            const double *tw, const Scal *stop_gate) {
  const size_t sh = (size_t)Lvl<R>::SIZE * sizeof(double);
  if (sh > 65536) lds_limit((const void *)k_dst2d<R>, sh);
  hipLaunchKernelGGL(k_dst2d<R>, dim3(n), dim3(kKT), sh, st, in, out, sin, sout, tw, 1.0 / sqrt(64.0 * R), stop_gate);
  return hipGetLastError();
}

hipError_t launch_dst2d(Ctx c, const double *in, double *out, long in_stride, long out_stride, const Scal *stop_gate) {
  const Plan *p = c.p;
  switch (p->L) {
    case 32: return run_dst2d<1>(c.st, p->n, in, out, in_stride, out_stride, p->tw, stop_gate);
    case 64: return run_dst2d<2>(c.st, p->n, in, out, in_stride, out_stride, p->tw, stop_gate);
    case 128: return run_dst2d<4>(c.st, p->n, in, out, in_stride, out_stride, p->tw, stop_gate);
    default: break;
  }
  return hipErrorInvalidValue;
}

KsP kslice_desc(const Plan *p, double *x, const double *bh) {
  KsP K{};
  K.N = p->N; K.n = p->n; K.m = p->m; K.ld = p->ld; K.L = p->L; K.scheme = p->scheme;
  K.blk0 = 0;
  K.theta = p->theta; K.tau = p->tau; K.h2inv = p->h2inv; K.scale = 1.0 / sqrt(2.0 * p->L);
  K.sqsigmin = p->sqsigmin;
  K.ax = p->ax; K.ay = p->ay; K.tw = p->tw;
  const bool f32 = p->pprec == SMR_FP32;
  for (int i = 0; i < 3; ++i) K.Z[i] = f32 ? (const void *)p->ZF[i] : (const void *)(i == 0 ? p->Z[0] : i == 1 ? p->Z[1] : p->Q);
  K.x = x; K.bh = bh; K.q = p->QX; K.kpart = p->part + kKsPartOffset; K.sc = p->sc;
  for (int i = 0; i < 4; ++i) K.y[i] = p->Y[i];
  return K;
}

hipError_t launch_kslice(Ctx c, int mode, int j, double *x, const double *bh) {
  const Plan *p = c.p;
  const KsP K = kslice_desc(p, x, bh);
  if (p->ks_split)
    return p->pprec == SMR_FP32 ? run_ks_split<1>(c.st, &K, nullptr, 1, p->n, mode, j)
                                : run_ks_split<0>(c.st, &K, nullptr, 1, p->n, mode, j);
  return p->pprec == SMR_FP32 ? run_ks_r<1>(c.st, p->L, &K, nullptr, 1, p->n, mode, j)
                              : run_ks_r<0>(c.st, p->L, &K, nullptr, 1, p->n, mode, j);
}

hipError_t launch_kslice_multi(hipStream_t st, const KsP *table, int ninst, int blocks, int L, int pprec, int mode,
                               int j, bool split) {
  if (split) {
    if (L != kKsN + 1) return hipErrorInvalidValue;
    return pprec == SMR_FP32 ? run_ks_split<1>(st, nullptr, table, ninst, blocks, mode, j)
                             : run_ks_split<0>(st, nullptr, table, ninst, blocks, mode, j);
  }
  return pprec == SMR_FP32 ? run_ks_r<1>(st, L, nullptr, table, ninst, blocks, mode, j)
                           : run_ks_r<0>(st, L, nullptr, table, ninst, blocks, mode, j);
}

}  // namespace smr
