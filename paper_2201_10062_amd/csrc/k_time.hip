// Time-axis sine transform (gfx950, FP64 or FP32 matrix cores).
//
// P_H^{-1} factorises as (S_n (x) U) diag(1/sigma) (S_n (x) U) (Sec. 3.1.1); along time the
// sine matrix S_n has no fast radix-2 form for the sizes used here (n + 1 = 65, 129, 257,
// 513), so it is applied as a dense GEMM on the matrix cores.  The reflection
// S[i][n+1-j] = (-1)^(i+1) S[i][j] folds it into two half-size blocks:
//   u_j = x_j + x_{n+1-j},  d_j = x_j - x_{n+1-j};  (S x)_odd = S_o u,  (S x)_even = S_e d,
// so S diag(w) S = B^T blockdiag(S_o^T D_o S_o, S_e^T D_e S_e) B with B the butterfly.
// Mode 0 applies S_n alone (P_theta); mode 1 applies S diag(1/sigma) S and accumulates
// <S x, diag(1/sigma) S x> (= gamma^2 by Parseval) per block.
//
// A block owns C consecutive columns (spatial points); its butterflied columns sit in
// LDS and its waves multiply them by the folded sine blocks (the fragments
// stream from L2 in MFMA-fragment order, two k-steps per load); the results go back to LDS,
// where the 1/sigma scaling and the final butterfly read them.
// PR 1 (mixed precision): the butterflied columns and the sine blocks are float32 and the
// GEMMs run on the float32 matrix cores with float32 accumulation; the 1/sigma scaling and the
// Parseval sum stay float64.  TI / TO: element types of the vectors in memory (float32 for the
// intermediates of a mixed-precision P^{-1}).
#include "smr_internal.h"
#include "mfma_tiles.h"

namespace smr {

namespace {

struct TimeP {
  int n, m, h1, h2;
  const void *So, *SoT, *Se, *SeT;     // folded sine blocks (fragment-pair order) in the GEMM precision
  const double *tcoef;                 // 4 per time mode: sigma = |(A + t B) + i (C + t D)|
  const double *tmu;                   // per column: t = tau * mu
};

// 1/sigma from a float reciprocal square root refined by two Newton steps in float64 (relative
// error ~1e-16; far cheaper than a float64 square root and division)
__device__ __forceinline__ double inv_sigma(const double *tc, int tmode, double t) {
  const double *c = tc + 4 * tmode;
  const double re = c[0] + t * c[1];
  const double im = c[2] + t * c[3];
  const double q = re * re + im * im;
  double r = (double)__frsqrt_rn((float)q);
  r = r * (1.5 - 0.5 * q * r * r);
  r = r * (1.5 - 0.5 * q * r * r);
  return r;
}

// sum over the NWV waves of the block, in a fixed order; valid in thread 0
template <int NWV>
__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NWV; ++w) s += red[w];
  return s;
}

// Both parities' GEMMs of one pass for the wave's tiles (tile = wave + 4 t, wave-uniform):
// ao[t] += Ao[r] * U[:, ct], ae[t] += Ae[r] * D[:, ct].  The tables hold the fragments of
// k-steps 2q and 2q+1 side by side per lane (one load fetches both); loads run two pairs
// ahead of the MFMAs (near the end they reload the last pair, unused, so that the loads need
// no branch).
template <int HP, int C, int PR>
__device__ __forceinline__ void pair_gemm(const typename Prec<PR>::T *__restrict__ Ao,
                                          const typename Prec<PR>::T *__restrict__ Ae,
                                          const typename Prec<PR>::T *U, const typename Prec<PR>::T *D,
                                          int wave, int lane,
                                          typename Prec<PR>::Acc (&ao)[((HP / 16) * (C / 16) + 3) / 4],
                                          typename Prec<PR>::Acc (&ae)[((HP / 16) * (C / 16) + 3) / 4]) {
  typedef typename Prec<PR>::T T;
  typedef typename std::conditional<PR == 0, double2, float2>::type T2;
  constexpr int LD = C + 1;
  constexpr int RT = HP / 16, CT = C / 16, NT = RT * CT, TPW = (NT + 3) / 4;
  constexpr int KS = HP / 4, KP = KS / 2;
  constexpr bool kAll = NT % 4 == 0;           // every wave owns TPW tiles
  const int bk = lane >> 4, bj = lane & 15;
  const T2 *__restrict__ Ao2 = reinterpret_cast<const T2 *>(Ao);
  const T2 *__restrict__ Ae2 = reinterpret_cast<const T2 *>(Ae);
  // a wave past the last tile reads row 0's fragments (valid, unused)
  size_t base[TPW];
  int boff[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + 4 * t;
    base[t] = (size_t)((kAll || tile < NT) ? tile / CT : 0) * KP * 64 + lane;
    boff[t] = bk * LD + 16 * (tile % CT) + bj;
  }
  T2 qo[TPW], qe[TPW], po[TPW], pe[TPW];     // pairs kp and kp + 1
  constexpr int K1 = KP > 1 ? 1 : 0;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    qo[t] = Ao2[base[t]];
    qe[t] = Ae2[base[t]];
    po[t] = Ao2[base[t] + (size_t)K1 * 64];
    pe[t] = Ae2[base[t] + (size_t)K1 * 64];
  }
#pragma unroll 1   // a rolled loop keeps the loads two pairs ahead (unrolled, they sink to their uses)
  for (int kp = 0; kp < KP; ++kp) {
    const int kn = kp + 2 < KP ? kp + 2 : KP - 1;
    T2 no[TPW], ne[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      no[t] = Ao2[base[t] + (size_t)kn * 64];
      ne[t] = Ae2[base[t] + (size_t)kn * 64];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = 2 * kp + h;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (kAll || wave + 4 * t < NT) {
          const T bu = U[4 * kk * LD + boff[t]];
          const T bd = D[4 * kk * LD + boff[t]];
          ao[t] = Prec<PR>::mfma(h ? qo[t].y : qo[t].x, bu, ao[t]);
          ae[t] = Prec<PR>::mfma(h ? qe[t].y : qe[t].x, bd, ae[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      qo[t] = po[t];
      qe[t] = pe[t];
      po[t] = no[t];
      pe[t] = ne[t];
    }
  }
}

// hp <= 32: both parities per k-step (each wave owns output tiles of both halves and keeps
// their accumulators; the final butterfly runs in registers).
template <int HP, int C, int MODE, int PR, typename TI, typename TO>
__global__ __launch_bounds__(256) void k_time_pair(TimeP tp, const TI *__restrict__ in, TO *__restrict__ out,
                                              double *__restrict__ part, const Scal *__restrict__ gate) {
  typedef typename Prec<PR>::T T;
  typedef typename Prec<PR>::Acc Acc;
  if (gate && gate->status != RUNNING) return;
  constexpr int LD = C + 1;                   // LDS row stride (doubles)
  constexpr int RT = HP / 16, CT = C / 16, NT = RT * CT;
  constexpr int TPW = (NT + 3) / 4;           // tiles per wave (per parity)
  extern __shared__ double lds_raw[];
  T *U = reinterpret_cast<T *>(lds_raw);      // [HP][LD] even-symmetric half (u)
  T *D = U + HP * LD;                         // [HP][LD] odd-symmetric half (d)
  const T *__restrict__ So = reinterpret_cast<const T *>(tp.So);
  const T *__restrict__ Se = reinterpret_cast<const T *>(tp.Se);
  const T *__restrict__ SoT = reinterpret_cast<const T *>(tp.SoT);
  const T *__restrict__ SeT = reinterpret_cast<const T *>(tp.SeT);
  __shared__ double red[4];

  // the wave index in a scalar register: the per-wave tile tests below are scalar branches
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col0 = blockIdx.x * C;
  const int n = tp.n, m = tp.m, h1 = tp.h1, h2 = tp.h2;

  // 1. butterfly load (zero padding rows and columns beyond m), eight elements per thread
  //    with all their loads issued before the LDS stores
  for (int e0 = tid; e0 < HP * C; e0 += 8 * 256) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      const int p = e / C, col = col0 + (e - p * C);
      const bool okc = e < HP * C && col < m;
      a[u] = okc && p < h1 ? (double)in[(size_t)p * m + col] : 0.0;
      b[u] = okc && p < h2 ? (double)in[(size_t)(n - 1 - p) * m + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      if (e >= HP * C) break;
      const int p = e / C, c = e - p * C;
      // p < h2: (u, d) = (a + b, a - b); odd n, p = h2: the middle level u = a, d = 0
      U[p * LD + c] = (T)(a[u] + b[u]);
      D[p * LD + c] = (T)(p < h2 ? a[u] - b[u] : 0.0);
    }
  }
  __syncthreads();

  const Acc zacc = {0, 0, 0, 0};
  Acc ao[TPW], ae[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) { ao[t] = zacc; ae[t] = zacc; }
  const int bk = lane >> 4, bj = lane & 15;

  // 2. first GEMM: [S_o u | S_e d] for this wave's tiles
  pair_gemm<HP, C, PR>(So, Se, U, D, wave, lane, ao, ae);

  if (MODE == 0) {
    // y_{2p} (odd modes) and y_{2p+1} (even modes), 0-based rows
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= NT) continue;
      const int r = tile / CT, ct = tile - r * CT;
      const int col = col0 + 16 * ct + bj;
      if (col >= m) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 16 * r + Prec<PR>::row(i, bk);
        if (p < h1) out[(size_t)(2 * p) * m + col] = (TO)ao[t][i];
        if (p < h2) out[(size_t)(2 * p + 1) * m + col] = (TO)ae[t][i];
      }
    }
    return;
  }

  // 3. scale by 1/sigma (time mode 2p+1 -> index 2p, 2p+2 -> 2p+1), Parseval partial
  double g2 = 0.0;
  __syncthreads();                            // every wave is done reading U, D
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= NT) continue;
    const int r = tile / CT, ct = tile - r * CT;
    const int cl = 16 * ct + bj, col = col0 + cl;
    const double tm = col < m ? tp.tmu[col] : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = 16 * r + Prec<PR>::row(i, bk);
      double so = 0.0, se = 0.0;
      if (col < m && p < h1) {
        const double a = (double)ao[t][i];
        so = a * inv_sigma(tp.tcoef, 2 * p, tm);
        g2 += a * so;
      }
      if (col < m && p < h2) {
        const double a = (double)ae[t][i];
        se = a * inv_sigma(tp.tcoef, 2 * p + 1, tm);
        g2 += a * se;
      }
      U[p * LD + cl] = (T)so;
      D[p * LD + cl] = (T)se;
    }
  }
  __syncthreads();

  // 4. second GEMM with the transposed blocks
#pragma unroll
  for (int t = 0; t < TPW; ++t) { ao[t] = zacc; ae[t] = zacc; }
  pair_gemm<HP, C, PR>(SoT, SeT, U, D, wave, lane, ao, ae);
  __syncthreads();   // all LDS reads done before any in-place global write of this block's columns

  // 5. output butterfly z_p = u'_p + d'_p, z_{n-1-p} = u'_p - d'_p (odd n: middle row once)
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= NT) continue;
    const int r = tile / CT, ct = tile - r * CT;
    const int col = col0 + 16 * ct + bj;
    if (col >= m) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = 16 * r + Prec<PR>::row(i, bk);
      const double a = (double)ao[t][i], b = (double)ae[t][i];
      if (p < h2) {
        out[(size_t)p * m + col] = (TO)(a + b);
        out[(size_t)(n - 1 - p) * m + col] = (TO)(a - b);
      } else if (p < h1) {
        out[(size_t)p * m + col] = (TO)a;
      }
    }
  }
  if (part) {
    const double s = block_sum<4>(g2, red);
    if (tid == 0) part[blockIdx.x] = s;
  }
}

// hp >= 64: one folded block per pass (fewer live accumulators), results through LDS.
// One block: C columns, all n levels; NW waves, all on the matrix cores (eight for hp >= 128,
// so that a CU holding a single block of the largest tiles still runs two waves per SIMD).
template <int HP, int C, int MODE, int PR, int NW, typename TI, typename TO>
__global__ __launch_bounds__(64 * NW) void k_time(TimeP tp, const TI *__restrict__ in,
                                                  TO *__restrict__ out, double *__restrict__ part,
                                                  const Scal *__restrict__ gate) {
  typedef typename Prec<PR>::T T;
  typedef typename Prec<PR>::Acc Acc;
  if (gate && gate->status != RUNNING) return;
  constexpr int NT = 64 * NW;
  constexpr int LD = C + 1;                   // LDS pitch
  constexpr int RPW = (HP / 16 + NW - 1) / NW, CT = C / 16;
  extern __shared__ double lds_raw[];
  T *U = reinterpret_cast<T *>(lds_raw);      // [HP][LD] even-symmetric half (u)
  T *D = U + HP * LD;                         // [HP][LD] odd-symmetric half (d)
  __shared__ double red[NW];
  // the 4 coefficients of every time mode, staged in LDS for the 1/sigma scaling where they
  // fit beside the two halves without lowering the blocks per CU (the float64 tiles up to
  // hp = 256); the scaling reads them per element
  constexpr int kHalves = 2 * HP * (C + 1) * (int)sizeof(T), kTcBytes = 8 * HP * (int)sizeof(double);
  constexpr int kLdsCU = 160 * 1024;
  constexpr bool kTcLds = MODE == 1 && kHalves + kTcBytes + 1024 <= kLdsCU &&
                          kLdsCU / (kHalves + kTcBytes + 1024) == kLdsCU / (kHalves + 1024);
  __shared__ double tcl[kTcLds ? 8 * HP : 1];
  const T *So = reinterpret_cast<const T *>(tp.So), *Se = reinterpret_cast<const T *>(tp.Se);
  const T *SoT = reinterpret_cast<const T *>(tp.SoT), *SeT = reinterpret_cast<const T *>(tp.SeT);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col0 = blockIdx.x * C;
  const int n = tp.n, m = tp.m, h1 = tp.h1, h2 = tp.h2;

  if (kTcLds)
    for (int e = tid; e < 4 * n; e += NT) tcl[e] = tp.tcoef[e];   // n <= 2 HP modes

  // 1. butterfly load (zero padding rows and columns beyond m), kBL elements per thread with
  //    all their loads issued before the LDS stores
  constexpr int kBL = 8;
  for (int e0 = tid; e0 < HP * C; e0 += kBL * NT) {
    double a[kBL], b[kBL];
#pragma unroll
    for (int u = 0; u < kBL; ++u) {
      const int e = e0 + u * NT;
      const int p = e / C, col = col0 + (e - p * C);
      const bool okc = e < HP * C && col < m;
      a[u] = okc && p < h1 ? (double)in[(size_t)p * m + col] : 0.0;
      b[u] = okc && p < h2 ? (double)in[(size_t)(n - 1 - p) * m + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBL; ++u) {
      const int e = e0 + u * NT;
      if (e >= HP * C) break;
      const int p = e / C, c = e - p * C;
      // p < h2: (u, d) = (a + b, a - b); odd n, p = h2: the middle level u = a, d = 0
      U[p * LD + c] = (T)(a[u] + b[u]);
      D[p * LD + c] = (T)(p < h2 ? a[u] - b[u] : 0.0);
    }
  }
  __syncthreads();

  // 2. [S_o u | S_e d], each result back to LDS once every wave is done reading its block.
  //    MODE 1 scales them by 1/sigma in registers on the way (time mode 2p+1 is row p of U,
  //    mode 2p+2 row p of D; padding rows and columns past m become zero) and accumulates the
  //    Parseval partial.
  const double *tc = kTcLds ? tcl : tp.tcoef;
  double g2 = 0.0;
  auto scale_acc = [&](Acc (&ac)[RPW][CT], int parity, int hlim) {
    constexpr int RT = HP / 16;
    const int wv = __builtin_amdgcn_readfirstlane(wave), bk = lane >> 4, bj = lane & 15;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wv + NW * i;
      if (r >= RT) continue;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int col = col0 + 16 * ct + bj;
        const bool okc = col < m;
        const double tm = tp.tmu[okc ? col : m - 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int p = 16 * r + Prec<PR>::row(q, bk);
          const double a = (double)ac[i][ct][q];
          double sv = 0.0;
          if (okc && p < hlim) {
            sv = a * inv_sigma(tc, 2 * p + parity, tm);
            g2 += a * sv;
          }
          ac[i][ct][q] = (T)sv;
        }
      }
    }
  };
  Acc acc[RPW][CT];
  gemm_tiles<HP, C, PR, NW>(So, U, wave, lane, acc);
  __syncthreads();
  if (MODE == 1) scale_acc(acc, 0, h1);
  store_acc<HP, C, PR, NW>(acc, U, wave, lane);
  gemm_tiles<HP, C, PR, NW>(Se, D, wave, lane, acc);
  __syncthreads();
  if (MODE == 1) scale_acc(acc, 1, h2);
  store_acc<HP, C, PR, NW>(acc, D, wave, lane);
  __syncthreads();

  if (MODE == 0) {
    // y_{2p} (odd modes) and y_{2p+1} (even modes), 0-based rows
    for (int e = tid; e < HP * C; e += NT) {
      const int p = e / C, c = e - p * C, col = col0 + c;
      if (col >= m) continue;
      if (p < h1) out[(size_t)(2 * p) * m + col] = (TO)U[p * LD + c];
      if (p < h2) out[(size_t)(2 * p + 1) * m + col] = (TO)D[p * LD + c];
    }
    return;
  }

  // 3. the transposed blocks
  gemm_tiles<HP, C, PR, NW>(SoT, U, wave, lane, acc);
  __syncthreads();
  store_acc<HP, C, PR, NW>(acc, U, wave, lane);
  gemm_tiles<HP, C, PR, NW>(SeT, D, wave, lane, acc);
  __syncthreads();
  store_acc<HP, C, PR, NW>(acc, D, wave, lane);
  __syncthreads();

  // 4. output butterfly z_p = u'_p + d'_p, z_{n-1-p} = u'_p - d'_p (odd n: middle row once)
  for (int e = tid; e < HP * C; e += NT) {
    const int p = e / C, c = e - p * C, col = col0 + c;
    if (col >= m) continue;
    const double a = (double)U[p * LD + c], b = (double)D[p * LD + c];
    if (p < h2) {
      out[(size_t)p * m + col] = (TO)(a + b);
      out[(size_t)(n - 1 - p) * m + col] = (TO)(a - b);
    } else if (p < h1) {
      out[(size_t)p * m + col] = (TO)a;
    }
  }
  if (part) {
    const double s = block_sum<NW>(g2, red);
    if (tid == 0) part[blockIdx.x] = s;
  }
}

template <int HP, int C, int PR, typename TI, typename TO>
hipError_t run_time(Ctx c, const TimeP &tp, const TI *in, TO *out, int mode, double *part, int *nb,
                    const Scal *gate) {
  const int blocks = (tp.m + C - 1) / C;
  if (nb) *nb = blocks;
  const size_t shmem = 2 * (size_t)HP * (C + 1) * sizeof(typename Prec<PR>::T);
  // hp >= 64: one folded block per pass on eight (hp >= 128) or four matrix-core waves; the
  // smaller paddings keep both parities per k-step (measured faster there)
  if constexpr (HP >= 64) {
    constexpr int NW = HP >= 128 ? 8 : 4;
    if (shmem > 65536) {
      (void)lds_limit((const void *)k_time<HP, C, 0, PR, NW, TI, TO>, shmem);
      (void)lds_limit((const void *)k_time<HP, C, 1, PR, NW, TI, TO>, shmem);
    }
    if (mode == 0)
      hipLaunchKernelGGL((k_time<HP, C, 0, PR, NW, TI, TO>), dim3(blocks), dim3(64 * NW), shmem, c.st, tp, in, out, part,
                         gate);
    else
      hipLaunchKernelGGL((k_time<HP, C, 1, PR, NW, TI, TO>), dim3(blocks), dim3(64 * NW), shmem, c.st, tp, in, out, part,
                         gate);
  } else {
    if (shmem > 65536) {
      (void)lds_limit((const void *)k_time_pair<HP, C, 0, PR, TI, TO>, shmem);
      (void)lds_limit((const void *)k_time_pair<HP, C, 1, PR, TI, TO>, shmem);
    }
    if (mode == 0)
      hipLaunchKernelGGL((k_time_pair<HP, C, 0, PR, TI, TO>), dim3(blocks), dim3(256), shmem, c.st, tp, in, out, part, gate);
    else
      hipLaunchKernelGGL((k_time_pair<HP, C, 1, PR, TI, TO>), dim3(blocks), dim3(256), shmem, c.st, tp, in, out, part, gate);
  }
  return hipGetLastError();
}

template <int PR, typename TI, typename TO>
hipError_t run_time_hp(Ctx c, const TimeP &tp, int hp, const TI *in, TO *out, int mode, double *part, int *nb,
                       const Scal *gate) {
  switch (hp) {
    case 16: return run_time<16, 32, PR>(c, tp, in, out, mode, part, nb, gate);
    case 32: return run_time<32, 32, PR>(c, tp, in, out, mode, part, nb, gate);
    case 64: return run_time<64, 32, PR>(c, tp, in, out, mode, part, nb, gate);
    case 128: return run_time<128, 32, PR>(c, tp, in, out, mode, part, nb, gate);
    case 256: return run_time<256, 32, PR>(c, tp, in, out, mode, part, nb, gate);
    case 512: return run_time<512, 16, PR>(c, tp, in, out, mode, part, nb, gate);
    default: break;
  }
  return hipErrorInvalidValue;
}

TimeP time_desc(const Plan *p, bool f32) {
  TimeP tp{p->n, p->m, p->h1, p->h2, p->So, p->SoT, p->Se, p->SeT, p->tcoef, p->tmu};
  if (f32) {
    tp.So = p->Sof; tp.SoT = p->SoTf; tp.Se = p->Sef; tp.SeT = p->SeTf;
  }
  return tp;
}

}  // namespace

hipError_t launch_time(Ctx c, const double *in, double *out, int mode, double *part, int *nb, const Scal *gate,
                       bool f32) {
  const Plan *p = c.p;
  if (f32 && p->pprec != SMR_FP32) return hipErrorInvalidValue;   // no float32 tables
  const TimeP tp = time_desc(p, f32);
  if (f32) return run_time_hp<1>(c, tp, p->hp, in, out, mode, part, nb, gate);
  return run_time_hp<0>(c, tp, p->hp, in, out, mode, part, nb, gate);
}

hipError_t launch_time_v(Ctx c, const void *in, bool in32, void *out, bool out32, int mode, double *part, int *nb,
                         const Scal *gate) {
  const Plan *p = c.p;
  if (p->pprec != SMR_FP32) return hipErrorInvalidValue;   // no float32 tables
  const TimeP tp = time_desc(p, true);
  if (in32 && out32) return run_time_hp<1>(c, tp, p->hp, (const float *)in, (float *)out, mode, part, nb, gate);
  if (!in32 && out32) return run_time_hp<1>(c, tp, p->hp, (const double *)in, (float *)out, mode, part, nb, gate);
  if (in32 && !out32) return run_time_hp<1>(c, tp, p->hp, (const float *)in, (double *)out, mode, part, nb, gate);
  return run_time_hp<1>(c, tp, p->hp, (const double *)in, (double *)out, mode, part, nb, gate);
}

}  // namespace smr
