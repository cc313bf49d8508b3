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
//      (v_0, w_0 and w_{-1} are zero by definition and never read, so nothing is cleared);
//      lagged search direction w_{j-1} and x_{j-1} (its coefficients need gamma_j, which
//      the previous launch produced);
//   B. true residual of x_{j-1}: ||Y b - (Y T)^ x||^2 partial;
//   C. z_{j+1} = S diag(1/sigma) S v_{j+1} on the FP64 matrix cores (two folded GEMMs),
//      gamma_{j+1}^2 = <v, z> by Parseval between them;
//   D. z_{j+1} stored, <(Y T)^ z_{j+1}, z_{j+1}> partial (gives delta_{j+1});
//   E. block partials, which every block of the next launch sums in a fixed order before
//      running the MINRES scalar recurrence (Givens rotation, convergence test) itself; above
//      kDirectTiles tiles a small launch between the two first sums them per tile group.
// The iterate x_{j-1} and its residual are final one launch after v_j, z_j: the stop test
// is the same (first iteration whose true residual is <= rtol), one launch later.
#include "k_spec_impl.h"

namespace smr {

// Launches of the 5-tap kernels (BDF3, BDF4), instantiated in k_spec5.hip.
hipError_t run_one_taps5(hipStream_t st, const SpecP &P, int pprec, int cols, int mode, int blocks, int hp, int jph,
                         int pmode);
hipError_t run_multi_taps5(hipStream_t st, const SpecP *table, int ninst, int blocks, int hp, int cols, int pprec,
                           int mode, int jph, int pmode);

namespace {

hipError_t run_one(hipStream_t st, const SpecP &P, int pprec, int cols, int mode, int blocks, int hp, int jph,
                   int pmode) {
  return (P.scheme == SMR_THETA || P.scheme == SMR_BDF2) ? run_one_taps<3>(st, P, pprec, cols, mode, blocks, hp, jph, pmode)
                     : run_one_taps5(st, P, pprec, cols, mode, blocks, hp, jph, pmode);
}

// The benign state a timing launch starts from: a running recurrence whose previous launch
// (slot 0) summed to ||r||^2 = 1, gamma^2 = 1, delta = 1/2 with no residual skipped.
__global__ void k_tune_state(Scal *__restrict__ sc, double *__restrict__ part, int npart,
                             double *__restrict__ kpart, int nkpart, Scal s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  if (i == 0) sc[0] = s;
  for (int k = i; k < npart; k += stride) part[k] = k == 0 || k == 2 ? 1.0 : k == 3 ? 0.5 : 0.0;
  if (kpart)
    for (int k = i; k < nkpart; k += stride) kpart[k] = 0.0;
}

}  // namespace

int spec_cols(const Plan *p) { return p->spec_c; }

int spec_cols_default(int hp) { return hp >= 256 ? 16 : 32; }

// 64-mode tiles at hp = 128 only with float32 transforms (two 128 x 65 float32 blocks in LDS;
// the float64 instance would hold one block per CU and spill)
bool spec_cols_ok(int hp, int cols, int pprec) {
  return cols == 16 || (cols == 32 && hp <= 128) || (cols == 64 && (hp <= 64 || (hp == 128 && pprec == SMR_FP32)));
}

SpecP spec_desc(const Plan *p, double *x, const double *bh, int cols) {
  SpecP P{};
  P.sqsigmin = p->sqsigmin;
  P.n = p->n; P.m = p->m; P.ld = p->ld; P.h1 = p->h1; P.h2 = p->h2; P.scheme = p->scheme; P.theta = p->theta;

  const int C = cols ? cols : p->spec_c;
  P.tiles = (p->m + C - 1) / C;
  P.tile0 = 0;
  const bool f32 = p->pprec == SMR_FP32;
  P.So = f32 ? (const void *)p->Sof : (const void *)p->So;
  P.SoT = f32 ? (const void *)p->SoTf : (const void *)p->SoT;
  P.Se = f32 ? (const void *)p->Sef : (const void *)p->Se;
  P.SeT = f32 ? (const void *)p->SeTf : (const void *)p->SeT;
  P.tcoef = p->tcoef; P.tmu = p->tmu;
  for (int i = 0; i < 3; ++i) P.Z[i] = f32 ? (void *)p->ZF[i] : (void *)(i == 0 ? p->Z[0] : i == 1 ? p->Z[1] : p->Q);
  P.V[0] = p->V[0]; P.V[1] = p->V[1]; P.W[0] = p->W[0]; P.W[1] = p->W[1];
  P.x = x; P.bh = bh; P.part = p->part; P.sc = p->sc;
  P.x0zero = 0; P.rtol = 0.0; P.maxit = 0;
  P.rtiles = P.tiles > kDirectTiles ? kPartGroups : 0;
  if (!p->const_coef) {
    P.qext = p->QX;
    P.kpart = p->part + kKsPartOffset;
    P.nks = p->ks_split ? p->n * kKsTiles : p->n;
  }
  return P;
}

size_t spec_part_doubles(int m) {
  const size_t tiles = (size_t)(m + 15) / 16;          // the narrow width has the most tiles
  const size_t need = 8 * tiles + 8 * (size_t)kPartGroups;
  return need > 16 * (size_t)kRedSlots ? need : 16 * (size_t)kRedSlots;
}

// Partial sums of fused launch j (slot j & 1) added per tile group: group g of kPartGroups
// owns a fixed, contiguous range of tiles, summed by one block in a fixed order.  Skipped
// when launch j found the solve stopped (it then wrote no partials, and the next launch does
// not read them).
__global__ __launch_bounds__(256) void k_part_reduce(double *__restrict__ part, int tiles, int slot,
                                                     const Scal *__restrict__ sc) {
  if (sc[slot].status != RUNNING) return;
  __shared__ double red[4][4];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int per = (tiles + kPartGroups - 1) / kPartGroups;
  const int b0 = g * per, b1 = min(tiles, b0 + per);
  const double *pp = part + (size_t)slot * 4 * tiles;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = b0 + tid; b < b1; b += 256)
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q] += pp[4 * (size_t)b + q];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int off = 32; off > 0; off >>= 1) t[q] += __shfl_xor(t[q], off, 64);
  if ((tid & 63) == 0)
    for (int q = 0; q < 4; ++q) red[q][tid >> 6] = t[q];
  __syncthreads();
  if (tid < 4) {
    double* out = part + 8 * (size_t)tiles + (size_t)slot * 4 * kPartGroups + 4 * (size_t)g;
    out[tid] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
  }
}

// mode of launch j - 1, whose partial sums launch j reduces (an early steady launch leaves
// them in the steady layout)
static int prev_mode(int mode, int j) { return mode == MODE_FIRST ? MODE_INIT : (j == 2 ? MODE_FIRST : MODE_STEADY); }

// launches 2 and 3 run the early variant of the steady iteration
static int launch_mode(int mode, int j) { return mode == MODE_STEADY && j < 4 ? MODE_EARLY : mode; }

hipError_t launch_spec(Ctx c, int mode, int j, double *x, const double *bh, bool x0zero, double rtol, int maxit) {
  const Plan *p = c.p;
  SpecP P = spec_desc(p, x, bh);
  P.x0zero = x0zero ? 1 : 0;
  P.rtol = rtol;
  P.maxit = maxit;
  const int jph = j % 6, pmode = prev_mode(mode, j);
  hipError_t e = run_one(c.st, P, p->pprec, p->spec_c, launch_mode(mode, j), P.tiles, p->hp, jph, pmode);
  if (e != hipSuccess || !P.rtiles) return e;
  hipLaunchKernelGGL(k_part_reduce, dim3(kPartGroups), dim3(256), 0, c.st, p->part, P.tiles, j & 1, p->sc);
  return hipGetLastError();
}

hipError_t spec_tune_state(const Plan *p, hipStream_t st, const SpecP &P) {
  (void)p;
  Scal s{};
  s.status = RUNNING; s.iter = 5; s.maxit = 1 << 30;
  s.gamma = s.gamma1 = s.gamma_new = s.zs = 1.0; s.delta = 0.5;
  s.c = s.c_old = 1.0; s.eta = 1.0; s.bnorm = 1.0; s.rtol = 0.0;   // never converges
  // the partials a launch with j = 7 reads (slot 0): per tile, or per tile group
  const int npart = 4 * (P.rtiles ? P.rtiles : P.tiles), nk = P.kpart ? 4 * P.nks : 0;
  double *tpart = P.rtiles ? P.part + 8 * (size_t)P.tiles : P.part;
  hipLaunchKernelGGL(k_tune_state, dim3((npart + 255) / 256), dim3(256), 0, st, P.sc, tpart, npart,
                     P.kpart ? const_cast<double *>(P.kpart) : nullptr, nk, s);
  return hipGetLastError();
}

hipError_t spec_tune(Plan *p, hipStream_t st) {
  if (!spec_cols_ok(p->hp, 32)) {
    p->spec_c = 16;
    return hipSuccess;
  }
  const std::vector<long> key{TUNE_SPEC_WIDTH, p->dim, p->hp, p->n, p->m, p->pprec, p->taps <= 3 ? 3 : 5,
                              p->const_coef ? 0 : 1};
  int cached = 0;
  if (tune_get(key, &cached)) {
    p->spec_c = cached;
    return hipSuccess;
  }
  hipError_t e = hipSuccess;
  const size_t vbytes = sizeof(double) * p->vlen;
  double *vecs[] = {p->V[0], p->V[1], p->Z[0], p->Z[1], p->W[0], p->W[1], p->Q, p->T1, p->T2, p->QX};
  for (double *v : vecs)
    if (v && e == hipSuccess) e = hipMemsetAsync(v, 0, vbytes, st);
  if (p->pprec == SMR_FP32)
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipMemsetAsync(p->ZF[i], 0, sizeof(float) * p->vlen, st);
  if (e != hipSuccess) return e;
  // a steady launch with j = 7 reads scalar and partial slot 0 and writes slot 1, so repeated
  // launches all start from the same state; 64-column tiles are a candidate at hp <= 64 (128 with float32 transforms)
  const int cand[3] = {32, 16, 64};
  const int ncand = spec_cols_ok(p->hp, 64, p->pprec) ? 3 : 2;
  float best[3] = {1e30f, 1e30f, 1e30f};
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
    for (int k = 0; k < ncand && e == hipSuccess; ++k) {
      p->spec_c = cand[k];
      const SpecP P = spec_desc(p, p->T1, p->T2);
      e = spec_tune_state(p, st, P);
      float ms = 0.0f;
      if (e == hipSuccess)
        e = tune_time(st, 6, [&]() {
          hipError_t r = run_one(st, P, p->pprec, cand[k], MODE_STEADY, P.tiles, p->hp, 1, MODE_STEADY);
          if (r == hipSuccess && P.rtiles)
            hipLaunchKernelGGL(k_part_reduce, dim3(kPartGroups), dim3(256), 0, st, p->part, P.tiles, 1, p->sc);
          return r == hipSuccess ? hipGetLastError() : r;
        }, &ms);
      if (e == hipSuccess) best[k] = std::min(best[k], ms);
    }
  // 32 stays unless another width is clearly (5%) faster; then the fastest
  int arg = 0;
  for (int k = 1; k < ncand; ++k)
    if (best[k] < 0.95f * best[0] && best[k] < best[arg]) arg = k;
  p->spec_c = cand[arg];
  if (e == hipSuccess) tune_put(key, p->spec_c);
  return e;
}

hipError_t launch_spec_multi(hipStream_t st, const SpecP *table, int ninst, int blocks, int hp, int cols, int pprec,
                             int taps, int mode, int j) {
  const int jph = j % 6, pmode = prev_mode(mode, j);
  mode = launch_mode(mode, j);
  return taps <= 3 ? run_multi_taps<3>(st, table, ninst, blocks, hp, cols, pprec, mode, jph, pmode)
                   : run_multi_taps5(st, table, ninst, blocks, hp, cols, pprec, mode, jph, pmode);
}

__global__ void k_gather_scal(const SpecP *__restrict__ table, int ninst, int slot, Scal *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) out[i] = table[i].sc[slot];
}

hipError_t launch_gather_scal(hipStream_t st, const SpecP *table, int ninst, int slot, Scal *out) {
  hipLaunchKernelGGL(k_gather_scal, dim3((ninst + 63) / 64), dim3(64), 0, st, table, ninst, slot, out);
  return hipGetLastError();
}

}  // namespace smr
