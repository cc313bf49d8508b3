// Matrix-core tiles of the folded time-axis sine transform (gfx950), shared by the fused
// sine-basis kernel and the physical-basis time transform.  A block holds C columns of a
// butterflied half (HP rows, LDS pitch C + 1); the NW matrix-core waves (wave 0..NW-1) each own
// the 16-row tiles r = wave + NW i, and one pass multiplies the block by one folded sine table.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace smr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

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

// GEMM of the NW matrix-core waves: for the 16-row tiles r = wave + NW i (i < RPW) and all
// CT column tiles, acc[i][ct] += A[r] * B[:, ct] over the k dimension, with B the LDS block.
// One A fragment feeds CT MFMAs.  The tables hold the fragments of k-steps 2q and 2q+1 side
// by side per lane, so one load fetches two k-steps; loads run two such pairs ahead, and the
// B fragments of the next k-step are read from LDS while the current one's MFMAs run.  The
// wave index is made wave-uniform (scalar), so the row test is a scalar branch, and it is
// dropped where NW divides the row tiles.
template <int HP, int C, int PR, int NW = 4>
__device__ __forceinline__ void gemm_tiles(const typename Prec<PR>::T *__restrict__ A,
                                           const typename Prec<PR>::T *Bs, int wave_in, int lane,
                                           typename Prec<PR>::Acc (&acc)[(HP / 16 + NW - 1) / NW][C / 16]) {
  typedef typename Prec<PR>::T T;
  typedef typename std::conditional<PR == 0, double2, float2>::type T2;
  constexpr int LD = C + 1;
  constexpr int RT = HP / 16, CT = C / 16, RPW = (RT + NW - 1) / NW;
  constexpr int KS = HP / 4, KP = KS / 2;         // k-steps, k-step pairs
  constexpr bool kAllRows = RT % NW == 0;
  const int wave = __builtin_amdgcn_readfirstlane(wave_in);
  const int bk = lane >> 4, bj = lane & 15;
  const T2 *__restrict__ A2 = reinterpret_cast<const T2 *>(A);
  const T2 zero2 = {T(0), T(0)};
  const typename Prec<PR>::Acc zacc = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[i][ct] = zacc;
  T2 q0[RPW], qn[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wave + NW * i;
    const bool ok = kAllRows || r < RT;
    q0[i] = ok ? A2[(size_t)r * KP * 64 + lane] : zero2;
    qn[i] = (ok && 1 < KP) ? A2[((size_t)r * KP + 1) * 64 + lane] : zero2;
  }
  const T *Bl = Bs + bk * LD + bj;
  T b[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) b[ct] = Bl[16 * ct];
  for (int kp = 0; kp < KP; ++kp) {
    T2 q1[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int r = wave + NW * i;
      q1[i] = qn[i];
      qn[i] = ((kAllRows || r < RT) && kp + 2 < KP) ? A2[((size_t)r * KP + kp + 2) * 64 + lane] : zero2;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kk = 2 * kp + h;
      T bn[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) bn[ct] = kk + 1 < KS ? Bl[4 * (kk + 1) * LD + 16 * ct] : T(0);
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        if (kAllRows || wave + NW * i < RT) {
          const T a = h ? q0[i].y : q0[i].x;
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[i][ct] = Prec<PR>::mfma(a, b[ct], acc[i][ct]);
        }
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) b[ct] = bn[ct];
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) q0[i] = q1[i];
  }
}

// Accumulator tiles of the NW matrix-core waves -> LDS rows, in the accumulator layout of
// the transform's precision.
template <int HP, int C, int PR, int NW = 4>
__device__ __forceinline__ void store_acc(const typename Prec<PR>::Acc (&acc)[(HP / 16 + NW - 1) / NW][C / 16],
                                          typename Prec<PR>::T *Dst, int wave, int lane) {
  constexpr int LD = C + 1;
  constexpr int RT = HP / 16, CT = C / 16, RPW = (RT + NW - 1) / NW;
  const int bk = lane >> 4, bj = lane & 15;
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = wave + NW * i;
    if (r >= RT) continue;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int cl = 16 * ct + bj;
#pragma unroll
      for (int q = 0; q < 4; ++q) Dst[(16 * r + Prec<PR>::row(q, bk)) * LD + cl] = acc[i][ct][q];
    }
  }
}

}  // namespace smr
