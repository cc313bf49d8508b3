// Time-axis sine transform (gfx950, FP64 matrix cores).
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
// LDS, the folded sine blocks stream from L2 in MFMA-fragment order, each of the 4
// waves owns a set of 16x16 output tiles of both parities, and the final butterfly is
// done in registers because a wave holds u' and d' of the same rows.
#include "smr_internal.h"

namespace smr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct TimeP {
  int n, m, h1, h2;
  const double *So, *SoT, *Se, *SeT;   // fragment order: [((r * HP/8 + kk/2) * 64 + lane) * 2 + kk%2]
  const double *tcoef;                 // 4 per time mode: sigma = |(A + t B) + i (C + t D)|
  const double *tmu;                   // per column: t = tau * mu
};

__device__ __forceinline__ double inv_sigma(const TimeP &tp, int tmode, double t) {
  const double *c = tp.tcoef + 4 * tmode;
  const double re = c[0] + t * c[1];
  const double im = c[2] + t * c[3];
  return 1.0 / sqrt(re * re + im * im);
}

__device__ __forceinline__ size_t frag_at(int r, int ks, int kk, int lane) {
  return (((size_t)r * (ks / 2) + kk / 2) * 64 + lane) * 2 + (kk & 1);
}

__device__ __forceinline__ double block_sum256(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < 4; ++w) s += red[w];
  return s;
}

template <int HP, int C, int MODE>
__global__ __launch_bounds__(256) void k_time(TimeP tp, const double *__restrict__ in, double *__restrict__ out,
                                              double *__restrict__ part, const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  constexpr int LD = C + 1;                   // LDS row stride (doubles)
  constexpr int RT = HP / 16, CT = C / 16, NT = RT * CT;
  constexpr int TPW = (NT + 3) / 4;           // tiles per wave (per parity)
  constexpr int KS = HP / 4;                  // k-steps
  extern __shared__ double lds[];
  double *U = lds;                            // [HP][LD] even-symmetric half (u)
  double *D = lds + HP * LD;                  // [HP][LD] odd-symmetric half (d)
  __shared__ double red[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col0 = blockIdx.x * C;
  const int n = tp.n, m = tp.m, h1 = tp.h1, h2 = tp.h2;

  // 1. butterfly load (zero padding rows and columns beyond m)
  for (int e = tid; e < HP * C; e += 256) {
    const int p = e / C, c = e - p * C;
    const int col = col0 + c;
    double u = 0.0, d = 0.0;
    if (col < m) {
      if (p < h2) {
        const double a = in[(size_t)p * m + col], b = in[(size_t)(n - 1 - p) * m + col];
        u = a + b;
        d = a - b;
      } else if (p < h1) {                   // odd n: middle level
        u = in[(size_t)p * m + col];
      }
    }
    U[p * LD + c] = u;
    D[p * LD + c] = d;
  }
  __syncthreads();

  d4 ao[TPW], ae[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) { ao[t] = d4{0, 0, 0, 0}; ae[t] = d4{0, 0, 0, 0}; }

  // Fragment layout of v_mfma_f64_16x16x4f64 (checked on gfx950): A[i][k] and B[k][j] sit in
  // lane i + 16k and j + 16k; accumulator register r of lane l holds D[4r + l/16][l%16].
  const int bk = lane >> 4, bj = lane & 15;

  // 2. first GEMM: [S_o u | S_e d] for this wave's tiles
  for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile < NT) {
        const int r = tile / CT, ct = tile - r * CT;
        const double bu = U[(4 * kk + bk) * LD + 16 * ct + bj];
        const double bd = D[(4 * kk + bk) * LD + 16 * ct + bj];
        const double au = tp.So[frag_at(r, KS, kk, lane)];
        const double ad = tp.Se[frag_at(r, KS, kk, lane)];
        ao[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, bu, ao[t], 0, 0, 0);
        ae[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad, bd, ae[t], 0, 0, 0);
      }
    }
  }

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
        const int p = 16 * r + 4 * i + bk;
        if (p < h1) out[(size_t)(2 * p) * m + col] = ao[t][i];
        if (p < h2) out[(size_t)(2 * p + 1) * m + col] = ae[t][i];
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
      const int p = 16 * r + 4 * i + bk;
      double so = 0.0, se = 0.0;
      if (col < m && p < h1) {
        const double w = inv_sigma(tp, 2 * p, tm);
        so = ao[t][i] * w;
        g2 += ao[t][i] * so;
      }
      if (col < m && p < h2) {
        const double w = inv_sigma(tp, 2 * p + 1, tm);
        se = ae[t][i] * w;
        g2 += ae[t][i] * se;
      }
      U[p * LD + cl] = so;
      D[p * LD + cl] = se;
    }
  }
  __syncthreads();

  // 4. second GEMM with the transposed blocks
#pragma unroll
  for (int t = 0; t < TPW; ++t) { ao[t] = d4{0, 0, 0, 0}; ae[t] = d4{0, 0, 0, 0}; }
  for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wave + 4 * t;
      if (tile < NT) {
        const int r = tile / CT, ct = tile - r * CT;
        const double bu = U[(4 * kk + bk) * LD + 16 * ct + bj];
        const double bd = D[(4 * kk + bk) * LD + 16 * ct + bj];
        const double au = tp.SoT[frag_at(r, KS, kk, lane)];
        const double ad = tp.SeT[frag_at(r, KS, kk, lane)];
        ao[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(au, bu, ao[t], 0, 0, 0);
        ae[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad, bd, ae[t], 0, 0, 0);
      }
    }
  }
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
      const int p = 16 * r + 4 * i + bk;
      if (p < h2) {
        out[(size_t)p * m + col] = ao[t][i] + ae[t][i];
        out[(size_t)(n - 1 - p) * m + col] = ao[t][i] - ae[t][i];
      } else if (p < h1) {
        out[(size_t)p * m + col] = ao[t][i];
      }
    }
  }
  if (part) {
    const double s = block_sum256(g2, red);
    if (tid == 0) part[blockIdx.x] = s;
  }
}

template <int HP, int C>
hipError_t run_time(Ctx c, const TimeP &tp, const double *in, double *out, int mode, double *part, int *nb,
                    const Scal *gate) {
  const int blocks = (tp.m + C - 1) / C;
  if (nb) *nb = blocks;
  const size_t shmem = 2 * (size_t)HP * (C + 1) * sizeof(double);
  if (shmem > 65536) {
    hipFuncSetAttribute((const void *)k_time<HP, C, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    hipFuncSetAttribute((const void *)k_time<HP, C, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  }
  if (mode == 0)
    hipLaunchKernelGGL((k_time<HP, C, 0>), dim3(blocks), dim3(256), shmem, c.st, tp, in, out, part, gate);
  else
    hipLaunchKernelGGL((k_time<HP, C, 1>), dim3(blocks), dim3(256), shmem, c.st, tp, in, out, part, gate);
  return hipGetLastError();
}

}  // namespace

int time_blocks(const Plan *p) {
  const int C = p->hp >= 512 ? 16 : 32;
  return (p->m + C - 1) / C;
}

hipError_t launch_time(Ctx c, const double *in, double *out, int mode, double *part, int *nb, const Scal *gate) {
  const Plan *p = c.p;
  TimeP tp{p->n, p->m, p->h1, p->h2, p->So, p->SoT, p->Se, p->SeT, p->tcoef, p->tmu};
  switch (p->hp) {
    case 16: return run_time<16, 32>(c, tp, in, out, mode, part, nb, gate);
    case 32: return run_time<32, 32>(c, tp, in, out, mode, part, nb, gate);
    case 64: return run_time<64, 32>(c, tp, in, out, mode, part, nb, gate);
    case 128: return run_time<128, 32>(c, tp, in, out, mode, part, nb, gate);
    case 256: return run_time<256, 32>(c, tp, in, out, mode, part, nb, gate);
    case 512: return run_time<512, 16>(c, tp, in, out, mode, part, nb, gate);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace smr
