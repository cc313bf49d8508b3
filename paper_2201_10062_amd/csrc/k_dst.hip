// Spatial sine transforms (gfx950), general form.  The orthonormal DST-I S_N (Sec. 3.1.1, S_n of
// eqn:matrix_tri_p with n -> N) along x (contiguous lines), y (stride-N lines) or, in 3D, z
// (stride-N^2 lines) of every time slice, for N + 1 = L a power of two.
//
// Method: two real lines a, b are packed as z = a + i b, extended oddly to length
// M = 2L (z_0 = z_L = 0, z_{2L-j} = -z_j) and transformed by one complex radix-2 FFT
// held in LDS (bit-reversed load, in-place decimation-in-time butterflies).  With
// Z = FFT(z): (S_N a)_k = -Im(Z_k) / sqrt(2L) and (S_N b)_k = Re(Z_k) / sqrt(2L).
// Each block owns `ppb` line pairs; all of its loads finish before any store, so the
// transform may run in place (with equal input and output slice strides).
#include "smr_internal.h"

namespace smr {

namespace {

struct DstP {
  int N, L, M, logM, m, nslices, ppb, tpp, dim, n;
  int rows;                   // lines per slice: 1 (1D), N (2D) or N^2 (3D)
  long sin, sout;             // slice strides of the input and the output (>= m)
  long nlines;
  double scale;               // 1/sqrt(2L)
  const double2 *tw;          // exp(-2 pi i t / M), t < M/2
  // optional diagonal division after the transform (Chebyshev inner preconditioner):
  // out /= ez[s] + ez[n + s] * abar * tmu_lap[q]
  const double *ez, *tmu_lap;
  double abar;
  int scale_mode;
};

__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Offset of element j of line r inside its slice, and the slice of line r.  Line i of a slice:
// x-line i (rows of N, i = z*N + y); y-line i = z*N + x; z-line i = y*N + x.
template <int DIR>
__device__ __forceinline__ size_t in_slice(const DstP &d, long r, int j, long &s) {
  s = r / d.rows;
  const int i = (int)(r - s * d.rows);
  const size_t N = d.N;
  if (DIR == 0) return (size_t)i * N + j;
  if (DIR == 1) return (size_t)(i / d.N) * N * N + (size_t)j * N + (size_t)(i % d.N);
  return (size_t)j * N * N + (size_t)i;
}

// TI, TO: element types of the input and output vectors (float32 intermediates of a
// mixed-precision P^{-1}); the FFT itself runs in float64.
template <int DIR, typename TI, typename TO>
__global__ __launch_bounds__(256) void k_dst(DstP d, const TI *__restrict__ in, TO *__restrict__ out,
                                             const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  extern __shared__ double2 X[];          // ppb * M complex values, then M/2 twiddles
  double2 *tw = X + (size_t)d.ppb * d.M;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int lpb = 2 * d.ppb;              // lines per block
  const long r0 = (long)blockIdx.x * lpb;

  for (int t = tid; t < d.M / 2; t += nthr) tw[t] = d.tw[t];
  // zero the two fixed points z_0 and z_L of every pair
  for (int p = tid; p < d.ppb; p += nthr) {
    X[(size_t)p * d.M + 0] = make_double2(0.0, 0.0);
    X[(size_t)p * d.M + bitrev(d.L, d.logM)] = make_double2(0.0, 0.0);
  }
  // load: element j of line c (c = 0..lpb-1) -> z_{j+1} of pair c/2, component c%2
  const int total = lpb * d.N;
  for (int e = tid; e < total; e += nthr) {
    int c, j;
    if (DIR == 0) { c = e / d.N; j = e - c * d.N; }
    else { j = e / lpb; c = e - j * lpb; }   // neighbouring threads: neighbouring lines
    const long r = r0 + c;
    double v = 0.0;
    if (r < d.nlines) {
      long s;
      const size_t q = in_slice<DIR>(d, r, j, s);
      v = (double)in[(size_t)s * d.sin + q];
    }
    double2 *Xp = X + (size_t)(c >> 1) * d.M;
    const int i1 = bitrev(j + 1, d.logM), i2 = bitrev(d.M - (j + 1), d.logM);
    if (c & 1) { Xp[i1].y = v; Xp[i2].y = -v; }
    else { Xp[i1].x = v; Xp[i2].x = -v; }
  }
  __syncthreads();
  // in-place radix-2 DIT butterflies; tpp threads per pair
  const int p = tid / d.tpp, tp = tid - p * d.tpp;
  for (int lh = 0; lh < d.logM; ++lh) {
    const int half = 1 << lh;
    if (p < d.ppb) {
      double2 *Xp = X + (size_t)p * d.M;
      for (int t = tp; t < d.M / 2; t += d.tpp) {
        const int k = t & (half - 1);
        const int i0 = ((t - k) << 1) + k, i1 = i0 + half;
        const double2 w = tw[k << (d.logM - 1 - lh)];
        const double2 b = cmul(Xp[i1], w), a = Xp[i0];
        Xp[i0] = make_double2(a.x + b.x, a.y + b.y);
        Xp[i1] = make_double2(a.x - b.x, a.y - b.y);
      }
    }
    __syncthreads();
  }
  // store: (S a)_k = -Im Z_{k+1} * scale, (S b)_k = Re Z_{k+1} * scale
  for (int e = tid; e < total; e += nthr) {
    int c, j;
    if (DIR == 0) { c = e / d.N; j = e - c * d.N; }
    else { j = e / lpb; c = e - j * lpb; }
    const long r = r0 + c;
    if (r >= d.nlines) continue;
    const double2 Z = X[(size_t)(c >> 1) * d.M + j + 1];
    double v = (c & 1) ? Z.x * d.scale : -Z.y * d.scale;
    long s;
    const size_t q = in_slice<DIR>(d, r, j, s);
    if (d.scale_mode == 1) v /= d.ez[s] + d.ez[d.n + s] * d.abar * d.tmu_lap[q];
    out[(size_t)s * d.sout + q] = (TO)v;
  }
}

DstP make_dst(const Plan *p, int dir, int nslices) {
  DstP d{};
  d.N = p->N;
  d.L = p->L;
  d.M = 2 * p->L;
  d.logM = p->logL + 1;
  d.m = p->m;
  d.n = p->n;
  d.dim = p->dim;
  d.nslices = nslices;
  d.rows = p->dim == 1 ? 1 : p->dim == 2 ? p->N : p->N * p->N;
  d.nlines = (long)nslices * d.rows;
  d.sin = d.sout = p->m;
  const int half = d.M / 2;
  if (dir == 0) {
    d.ppb = half >= 256 ? 1 : 256 / half;
  } else {
    d.ppb = d.M <= 512 ? 8 : 4;
  }
  if (d.ppb > (d.nlines + 1) / 2) d.ppb = (int)((d.nlines + 1) / 2);
  if (d.ppb < 1) d.ppb = 1;
  d.tpp = 256 / d.ppb;
  if (d.tpp < 1) d.tpp = 1;
  d.scale = 1.0 / sqrt(2.0 * p->L);
  d.tw = reinterpret_cast<const double2 *>(p->tw);
  d.ez = p->ez;
  d.tmu_lap = p->tmu_lap;
  d.abar = p->abar;
  d.scale_mode = 0;
  return d;
}

template <typename TI, typename TO>
hipError_t run_dst_t(Ctx c, int dir, const TI *in, TO *out, int nslices, int scale_mode, const Scal *gate,
                     long in_stride, long out_stride) {
  if (dir < 0 || dir >= c.p->dim) return hipErrorInvalidValue;
  DstP d = make_dst(c.p, dir, nslices);
  d.scale_mode = scale_mode;
  if (in_stride) d.sin = in_stride;
  if (out_stride) d.sout = out_stride;
  const long lpb = 2L * d.ppb;
  const long nblocks = (d.nlines + lpb - 1) / lpb;
  const size_t shmem = ((size_t)d.ppb * d.M + d.M / 2) * sizeof(double2);
  const void *f = dir == 0 ? (const void *)k_dst<0, TI, TO> : dir == 1 ? (const void *)k_dst<1, TI, TO>
                                                                       : (const void *)k_dst<2, TI, TO>;
  if (shmem > 65536) {
    hipError_t e = lds_limit(f, shmem);
    if (e != hipSuccess) return e;
  }
  if (dir == 0)
    hipLaunchKernelGGL((k_dst<0, TI, TO>), dim3((unsigned)nblocks), dim3(256), shmem, c.st, d, in, out, gate);
  else if (dir == 1)
    hipLaunchKernelGGL((k_dst<1, TI, TO>), dim3((unsigned)nblocks), dim3(256), shmem, c.st, d, in, out, gate);
  else
    hipLaunchKernelGGL((k_dst<2, TI, TO>), dim3((unsigned)nblocks), dim3(256), shmem, c.st, d, in, out, gate);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dst_v(Ctx c, int dir, const void *in, bool in32, void *out, bool out32, int nslices,
                        int scale_mode, const Scal *gate, long in_stride, long out_stride, bool col16) {
  // 2D with N + 1 in {32, ..., 256}: line tiles through the register FFT
  if (dst_tile_supported(c.p))
    return launch_dst_tile(c, dir, in, in32, out, out32, nslices, scale_mode, gate, in_stride, out_stride, col16);
  if (!in32 && !out32)
    return run_dst_t(c, dir, (const double *)in, (double *)out, nslices, scale_mode, gate, in_stride, out_stride);
  if (!in32 && out32)
    return run_dst_t(c, dir, (const double *)in, (float *)out, nslices, scale_mode, gate, in_stride, out_stride);
  if (in32 && out32)
    return run_dst_t(c, dir, (const float *)in, (float *)out, nslices, scale_mode, gate, in_stride, out_stride);
  return run_dst_t(c, dir, (const float *)in, (double *)out, nslices, scale_mode, gate, in_stride, out_stride);
}

hipError_t launch_dst(Ctx c, int dir, const double *in, double *out, int nslices, int scale_mode,
                      const Scal *gate, long in_stride, long out_stride) {
  return launch_dst_v(c, dir, in, false, out, false, nslices, scale_mode, gate, in_stride, out_stride);
}

}  // namespace smr
