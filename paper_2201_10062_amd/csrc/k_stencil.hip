// Space-time stencil kernels (gfx950): the all-at-once matvec Y T x, right-hand side
// assembly, their adjoints, the coefficient gradient, MINRES vector updates, dot
// products and the device-side MINRES scalar recurrence.
//
// Every reduction is deterministic: each block writes one partial sum, and a single
// block later adds the partials in a fixed order.
#include "smr_internal.h"

#include <algorithm>
#include <cmath>

namespace smr {

namespace {

constexpr int kTX = 64, kTY = 4;      // 2D / 3D tile: 64 x-points by 4 rows (y, or z*N + y) per block
constexpr int kT1 = 256;              // 1D tile

struct SP {                           // stencil parameters passed by value
  int dim, N, n, m, scheme, taps;
  double tau, theta, h2inv;
  double tc[5];                       // time-difference coefficients of the levels t .. t-4
  const double *ax, *ay, *az;
};

inline SP make_sp(const Plan *p) {
  SP s{p->dim, p->N, p->n, p->m, p->scheme, p->taps, p->tau, p->theta, p->h2inv, {}, p->ax, p->ay, p->az};
  for (int k = 0; k < 5; ++k) s.tc[k] = p->tcf[k];
  return s;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  // wave64 butterfly, then across the (<= 16) waves through LDS
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x + threadIdx.y * blockDim.x;
  const int wave = lane >> 6;
  const int nw = (blockDim.x * blockDim.y + 63) >> 6;
  __syncthreads();
  if ((lane & 63) == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (lane == 0)
    for (int w = 0; w < nw; ++w) s += red[w];
  return s;   // valid in thread 0 only
}

// u = c0*x0 + c1*x1 (x1 may be null) at flat index q (T: the vectors' element type)
template <typename T>
__device__ __forceinline__ double comb(const T *__restrict__ x0, double c0, const T *__restrict__ x1, double c1,
                                       int q) {
  double v = c0 * (double)x0[q];
  if (x1) v += c1 * (double)x1[q];
  return v;
}

// (K u)(j, i) with u = c0*x0 + c1*x1 on one slice; zero Dirichlet values outside.  Row j is y
// in 2D and z*N + y in 3D (the 7-point stencil adds the two z neighbours N^2 apart).
template <typename T>
__device__ __forceinline__ double Kapply(const SP &s, const T *__restrict__ x0, double c0, const T *__restrict__ x1,
                                         double c1, int j, int i) {
  const int N = s.N;
  if (s.dim == 1) {
    const double uc = comb(x0, c0, x1, c1, i);
    const double uw = i > 0 ? comb(x0, c0, x1, c1, i - 1) : 0.0;
    const double ue = i < N - 1 ? comb(x0, c0, x1, c1, i + 1) : 0.0;
    return s.h2inv * (s.ax[i] * (uc - uw) + s.ax[i + 1] * (uc - ue));
  }
  const int y = s.dim == 3 ? j % N : j, z = s.dim == 3 ? j / N : 0;
  const int q = j * N + i;
  const double uc = comb(x0, c0, x1, c1, q);
  const double uw = i > 0 ? comb(x0, c0, x1, c1, q - 1) : 0.0;
  const double ue = i < N - 1 ? comb(x0, c0, x1, c1, q + 1) : 0.0;
  const double us = y > 0 ? comb(x0, c0, x1, c1, q - N) : 0.0;
  const double un = y < N - 1 ? comb(x0, c0, x1, c1, q + N) : 0.0;
  const double aw = s.ax[j * (N + 1) + i], ae = s.ax[j * (N + 1) + i + 1];
  const int ya = (z * (N + 1) + y) * N + i;
  const double as = s.ay[ya], an = s.ay[ya + N];
  double v = aw * (uc - uw) + ae * (uc - ue) + as * (uc - us) + an * (uc - un);
  if (s.dim == 3) {
    const int NN = N * N;
    const double ud = z > 0 ? comb(x0, c0, x1, c1, q - NN) : 0.0;
    const double uu = z < N - 1 ? comb(x0, c0, x1, c1, q + NN) : 0.0;
    v += s.az[q] * (uc - ud) + s.az[q + NN] * (uc - uu);
  }
  return s.h2inv * v;
}

// (T x)_k at spatial point (j, i): theta scheme x_k - x_{k-1} + tau K(theta x_k + (1-theta) x_{k-1});
// BDF-l sum_{r <= l} alpha_r x_{k-r} + tau K x_k.
__device__ __forceinline__ double Tapply(const SP &s, const double *__restrict__ x, int k, int j, int i) {
  const int m = s.m;
  const int q = (s.dim == 1) ? i : j * s.N + i;
  const double *xk = x + (size_t)k * m;
  const double *xk1 = k >= 1 ? xk - m : nullptr;
  if (s.scheme == SMR_THETA) {
    double v = xk[q] - (xk1 ? xk1[q] : 0.0);
    return v + s.tau * Kapply<double>(s, xk, s.theta, xk1, 1.0 - s.theta, j, i);
  }
  double v = 0.0;
  for (int r = 0; r < s.taps && r <= k; ++r) v += s.tc[r] * xk[q - (ptrdiff_t)r * m];
  return v + s.tau * Kapply<double>(s, xk, 1.0, nullptr, 0.0, j, i);
}

struct TileInfo {
  int ni, nj, ntiles;
};

// rows of one slice: y (2D) or z*N + y (3D)
__host__ __device__ inline int rows_of(int dim, int N) { return dim == 1 ? 1 : dim == 2 ? N : N * N; }

inline TileInfo tiles_of(const Plan *p, int nslices) {
  TileInfo t;
  if (p->dim == 1) {
    t.ni = (p->N + kT1 - 1) / kT1;
    t.nj = 1;
  } else {
    t.ni = (p->N + kTX - 1) / kTX;
    t.nj = (rows_of(p->dim, p->N) + kTY - 1) / kTY;
  }
  t.ntiles = t.ni * t.nj * nslices;
  return t;
}

inline dim3 block_of(const Plan *p) { return p->dim == 1 ? dim3(kT1, 1) : dim3(kTX, kTY); }

__device__ __forceinline__ bool tile_point(int t, int ni, int nj, int N, int dim, int &k, int &j, int &i) {
  const int it = t % ni;
  const int r = t / ni;
  const int jt = r % nj;
  k = r / nj;
  if (dim == 1) {
    i = it * kT1 + threadIdx.x;
    j = 0;
  } else {
    i = it * kTX + threadIdx.x;
    j = jt * kTY + threadIdx.y;
  }
  return i < N && j < rows_of(dim, N);
}

// MODE 0: y = Y T (xs x), partial <y, xs x>.   MODE 1: r = Y rhs - Y T x (written to y
// if y != null), partials ||r||^2 (slot 0) and ||rhs||^2 (slot 1).
// A block owns a spatial tile (64 x 4 points in 2D, 256 in 1D) and a run of kr time levels;
// each thread marches up its run keeping the previous levels and K x_{k-1} in registers, so
// that one 5-point stencil per level serves both terms of the theta scheme (K is linear).
struct MarchP {
  int ni, nj, nkc, kr;        // spatial tiles per axis, time runs, levels per run
};

template <int MODE>
__global__ __launch_bounds__(256) void k_apply_YT(SP s, MarchP mp, const double *__restrict__ x,
                                                  const double *__restrict__ d_xscale, double *__restrict__ y,
                                                  const double *__restrict__ rhs, double *__restrict__ part,
                                                  const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  __shared__ double red[16];
  const double xs = d_xscale ? *d_xscale : 1.0;
  const int N = s.N, m = s.m;
  const int b = blockIdx.x;
  const int it = b % mp.ni, jt = (b / mp.ni) % mp.nj, kc = b / (mp.ni * mp.nj);
  const int i = s.dim == 1 ? it * kT1 + threadIdx.x : it * kTX + threadIdx.x;
  const int j = s.dim == 1 ? 0 : jt * kTY + threadIdx.y;
  const bool ok = i < N && j < rows_of(s.dim, N);
  const int k0 = kc * mp.kr, k1 = min(s.n, k0 + mp.kr);
  double acc0 = 0.0, acc1 = 0.0;
  if (ok) {
    const int q = s.dim == 1 ? i : j * N + i;
    const int jy = s.dim == 3 ? j % N : j, jz = s.dim == 3 ? j / N : 0;
    const int NN = N * N;
    // neighbour offsets (0 = outside: the Dirichlet value 0) and face coefficients
    const bool hw = i > 0, he = i < N - 1, hs = s.dim >= 2 && jy > 0, hn = s.dim >= 2 && jy < N - 1;
    const bool hd = s.dim == 3 && jz > 0, hu = s.dim == 3 && jz < N - 1;
    double aw, ae, as = 0.0, an = 0.0, ad = 0.0, au = 0.0;
    if (s.dim == 1) {
      aw = s.ax[i];
      ae = s.ax[i + 1];
    } else {
      aw = s.ax[j * (N + 1) + i];
      ae = s.ax[j * (N + 1) + i + 1];
      const int ya = (jz * (N + 1) + jy) * N + i;
      as = s.ay[ya];
      an = s.ay[ya + N];
      if (s.dim == 3) {
        ad = s.az[q];
        au = s.az[q + NN];
      }
    }
    auto kx = [&](const double *xl, double &c) {   // c = x_l at q, returns (K x_l) at q
      c = xl[q];
      const double uw = hw ? xl[q - 1] : 0.0, ue = he ? xl[q + 1] : 0.0;
      const double us = hs ? xl[q - N] : 0.0, un = hn ? xl[q + N] : 0.0;
      const double ud = hd ? xl[q - NN] : 0.0, uu = hu ? xl[q + NN] : 0.0;
      return s.h2inv * (aw * (c - uw) + ae * (c - ue) + as * (c - us) + an * (c - un) + ad * (c - ud) + au * (c - uu));
    };
    double xp[4] = {0.0, 0.0, 0.0, 0.0};           // x_{k-1} .. x_{k-4}
    double kx1 = 0.0;                              // (K x)_{k-1} (theta method)
    if (k0 >= 1 && s.scheme == SMR_THETA) kx1 = kx(x + (size_t)(k0 - 1) * m, xp[0]);
    if (s.scheme != SMR_THETA)
      for (int r = 1; r < s.taps; ++r)
        if (k0 >= r) xp[r - 1] = x[(size_t)(k0 - r) * m + q];
    for (int k = k0; k < k1; ++k) {
      double x0;
      const double kx0 = kx(x + (size_t)k * m, x0);
      double tv;
      if (s.scheme == SMR_THETA) {
        tv = x0 - xp[0] + s.tau * (s.theta * kx0 + (1.0 - s.theta) * kx1);
      } else {
        tv = s.tc[0] * x0 + s.tau * kx0;
#pragma unroll
        for (int r = 1; r < 5; ++r) tv += s.tc[r] * xp[r - 1];   // zero past the scheme's taps
      }
      const size_t o = (size_t)(s.n - 1 - k) * m + q;   // Y: time level k lands at n-1-k
      if (MODE == 0) {
        const double val = xs * tv;
        if (y) y[o] = val;
        acc0 += val * (xs * x[o]);
      } else {
        const double bk = rhs[(size_t)k * m + q];
        const double r = bk - tv;
        if (y) y[o] = r;
        acc0 += r * r;
        acc1 += bk * bk;
      }
      xp[3] = xp[2];
      xp[2] = xp[1];
      xp[1] = xp[0];
      xp[0] = x0;
      kx1 = kx0;
    }
  }
  if (part) {
    const double s0 = block_sum(acc0, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = s0;
    if (MODE == 1) {
      const double s1 = block_sum(acc1, red);
      if (threadIdx.x == 0 && threadIdx.y == 0) part[kRedSlots + blockIdx.x] = s1;
    }
  }
}

__global__ __launch_bounds__(256) void k_build_rhs(SP s, TileInfo ti, const double *__restrict__ f,
                                                   const double *__restrict__ u0, double *__restrict__ b) {
  for (int t = blockIdx.x; t < ti.ntiles; t += gridDim.x) {
    int k, j, i;
    if (!tile_point(t, ti.ni, ti.nj, s.N, s.dim, k, j, i)) continue;
    const int q = (s.dim == 1) ? i : j * s.N + i;
    double v = s.theta * s.tau * f[(size_t)(k + 1) * s.m + q] + (1.0 - s.theta) * s.tau * f[(size_t)k * s.m + q];
    if (k == 0 && u0) v += u0[q] - (1.0 - s.theta) * s.tau * Kapply<double>(s, u0, 1.0, nullptr, 0.0, j, i);
    b[(size_t)k * s.m + q] = v;
  }
}

// grad f^(k) for k = 0..n (nslices = n+1), grad u0 on level 0.
__global__ __launch_bounds__(256) void k_rhs_adjoint(SP s, TileInfo ti, const double *__restrict__ lam,
                                                     double *__restrict__ gf, double *__restrict__ gu0) {
  for (int t = blockIdx.x; t < ti.ntiles; t += gridDim.x) {
    int k, j, i;
    if (!tile_point(t, ti.ni, ti.nj, s.N, s.dim, k, j, i)) continue;
    const int q = (s.dim == 1) ? i : j * s.N + i;
    double v = 0.0;
    if (k >= 1) v += s.theta * s.tau * lam[(size_t)(k - 1) * s.m + q];
    if (k <= s.n - 1) v += (1.0 - s.theta) * s.tau * lam[(size_t)k * s.m + q];
    gf[(size_t)k * s.m + q] = v;
    if (k == 0 && gu0) gu0[q] = lam[q] - (1.0 - s.theta) * s.tau * Kapply<double>(s, lam, 1.0, nullptr, 0.0, j, i);
  }
}

// One thread per face: grad a_e = -(tau/h^2) sum_k (D_e lam_k)(D_e ut_k).
__global__ __launch_bounds__(256) void k_grad_faces(SP s, const double *__restrict__ u,
                                                    const double *__restrict__ u0,
                                                    const double *__restrict__ lam, double *__restrict__ gax,
                                                    double *__restrict__ gay) {
  const int N = s.N, m = s.m;
  const int nx = (s.dim == 1) ? N + 1 : N * (N + 1);
  const int ny = (s.dim == 1) ? 0 : (N + 1) * N;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx + ny) return;
  int qa = -1, qb = -1;   // interior indices of the two nodes (-1 = boundary)
  if (e < nx) {
    if (s.dim == 1) {
      const int i = e;
      qa = i - 1;
      qb = i < N ? i : -1;
    } else {
      const int j = e / (N + 1), i = e % (N + 1);
      qa = i >= 1 ? j * N + i - 1 : -1;
      qb = i < N ? j * N + i : -1;
    }
  } else {
    const int f = e - nx;
    const int j = f / N, i = f % N;
    qa = j >= 1 ? (j - 1) * N + i : -1;
    qb = j < N ? j * N + i : -1;
  }
  const double th = (s.scheme == SMR_THETA) ? s.theta : 1.0;
  double acc = 0.0;
  for (int k = 0; k < s.n; ++k) {
    const double *lk = lam + (size_t)k * m;
    const double *uk = u + (size_t)k * m;
    const double *up = k >= 1 ? uk - m : u0;    // u_{k-1}, u_{-1} = u0 (may be null)
    const double la = qa >= 0 ? lk[qa] : 0.0, lb = qb >= 0 ? lk[qb] : 0.0;
    double ua = qa >= 0 ? th * uk[qa] : 0.0, ub = qb >= 0 ? th * uk[qb] : 0.0;
    if (th != 1.0 && up) {
      if (qa >= 0) ua += (1.0 - th) * up[qa];
      if (qb >= 0) ub += (1.0 - th) * up[qb];
    }
    acc += (lb - la) * (ub - ua);
  }
  const double g = -s.tau * s.h2inv * acc;
  if (e < nx) gax[e] = g;
  else gay[e - nx] = g;
}

// Nodal gradient: half the sum of the gradients of the faces touching each node.
__global__ __launch_bounds__(256) void k_grad_nodal(int dim, int N, const double *__restrict__ gax,
                                                    const double *__restrict__ gay, double *__restrict__ gn) {
  const int G = N + 2;
  const int total = dim == 1 ? G : G * G;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  double v = 0.0;
  if (dim == 1) {
    const int I = idx;           // face i joins nodes i and i+1
    if (I - 1 >= 0 && I - 1 <= N) v += gax[I - 1];
    if (I <= N) v += gax[I];
  } else {
    const int J = idx / G, I = idx % G;
    // x-face (j, i) joins nodes (J=j+1, I=i) and (J=j+1, I=i+1)
    if (J >= 1 && J <= N) {
      if (I <= N) v += gax[(J - 1) * (N + 1) + I];
      if (I >= 1) v += gax[(J - 1) * (N + 1) + I - 1];
    }
    // y-face (j, i) joins nodes (J=j, I=i+1) and (J=j+1, I=i+1)
    if (I >= 1 && I <= N) {
      if (J <= N) v += gay[J * N + I - 1];
      if (J >= 1) v += gay[(J - 1) * N + I - 1];
    }
  }
  gn[idx] = 0.5 * v;
}

// v_{j+1} = q - va v_j - vb v_{j-1}, written over v_{j-1}.
__global__ __launch_bounds__(256) void k_vupdate(size_t len, const double *__restrict__ q,
                                                 const double *__restrict__ v, double *__restrict__ vo,
                                                 const Scal *__restrict__ sc) {
  if (sc->status != RUNNING) return;
  const double va = sc->va, vb = sc->vb;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    vo[e] = q[e] - va * v[e] - vb * vo[e];
}

// w_j = (zs z - a3 w_{j-2} - a2 w_{j-1}) / a1 written over w_{j-2}; x += ceta w_j.
__global__ __launch_bounds__(256) void k_wxupdate(size_t len, const double *__restrict__ z,
                                                  double *__restrict__ wo, const double *__restrict__ w,
                                                  double *__restrict__ x, const Scal *__restrict__ sc) {
  if (sc->status != RUNNING) return;
  const double zs = sc->zs, a1 = sc->a1, a2 = sc->a2, a3 = sc->a3, ce = sc->ceta;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
    const double wn = (zs * z[e] - a3 * wo[e] - a2 * w[e]) / a1;
    wo[e] = wn;
    x[e] += ce * wn;
  }
}

__global__ __launch_bounds__(256) void k_dot(size_t len, const double *__restrict__ a, const double *__restrict__ b,
                                             double *__restrict__ part, const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    acc += a[e] * b[e];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_zero_int(int count, int *__restrict__ x) {
  for (int e = threadIdx.x; e < count; e += blockDim.x) x[e] = 0;
}

__global__ __launch_bounds__(256) void k_scale_copy(int n, int m, const double *__restrict__ in,
                                                    double *__restrict__ out, double s, int flip) {
  const size_t len = (size_t)n * m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
    size_t src = e;
    if (flip) {
      const size_t k = e / m, q = e - k * m;
      src = (size_t)(n - 1 - k) * m + q;
    }
    out[e] = s * in[src];
  }
}

__global__ __launch_bounds__(256) void k_zero(size_t len, double *__restrict__ x) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

// Sum nb partials in a fixed order (one block).
__device__ double fixed_sum(const double *part, int nb, double *red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[i];
  return block_sum(acc, red);
}

// The MINRES scalar recurrence, one block.  stage 0: initialise from ||r0||^2, ||b||^2 and
// gamma_1^2; stage 1: delta; stage 2: gamma_{j+1} and the Givens update; stage 3: true
// residual test and the shift of gamma.
__global__ __launch_bounds__(256) void k_scalar_step(int stage, Scal *sc, const double *__restrict__ part,
                                                     int nb, const double *__restrict__ part2, int nb2) {
  __shared__ double red[16];
  __shared__ double tot[3];
  if (stage != 0 && sc->status != RUNNING) return;
  const double s0 = fixed_sum(part, nb, red);
  if (threadIdx.x == 0) tot[0] = s0;
  if (stage == 0) {
    const double s1 = fixed_sum(part + kRedSlots, nb, red);
    if (threadIdx.x == 0) tot[1] = s1;
  }
  if (part2) {
    const double s2 = fixed_sum(part2, nb2, red);
    if (threadIdx.x == 0) tot[2] = s2;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (stage == 0) {
    const double r2 = tot[0], b2 = tot[1], g2 = tot[2];
    sc->bnorm = sqrt(b2);
    sc->iter = 0;
    sc->exact = 0;
    sc->status = RUNNING;
    if (b2 == 0.0) { sc->relres = 0.0; sc->status = DONE_CONV; return; }   // x = 0 is exact
    sc->relres = sqrt(r2) / sc->bnorm;
    if (sc->relres <= sc->rtol) { sc->status = DONE_CONV; return; }
    if (!(g2 > 0.0) || !isfinite(g2)) { sc->status = DONE_NOTSPD; return; }
    const double g = sqrt(g2);
    sc->gamma = g; sc->gamma1 = g; sc->gamma_old = 1.0;
    sc->eta = g; sc->c = sc->c_old = 1.0; sc->s = sc->s_old = 0.0;
    sc->zs = 1.0 / g;
    if (sc->maxit <= 0) sc->status = DONE_MAXIT;
  } else if (stage == 1) {
    sc->delta = tot[0];
    sc->va = sc->delta / sc->gamma;
    sc->vb = sc->gamma / sc->gamma_old;
  } else if (stage == 2) {
    const double g2 = part2 ? tot[2] : tot[0];
    if (g2 < 0.0 || !isfinite(g2)) { sc->status = DONE_NOTSPD; return; }
    const double gn = sqrt(g2);
    const double a0 = sc->c * sc->delta - sc->c_old * sc->s * sc->gamma;
    const double a1 = sqrt(a0 * a0 + gn * gn);
    const double a2 = sc->s * sc->delta + sc->c_old * sc->c * sc->gamma;
    const double a3 = sc->s_old * sc->gamma;
    if (a1 == 0.0) { sc->status = DONE_BREAKDOWN; return; }
    sc->c_old = sc->c; sc->c = a0 / a1;
    sc->s_old = sc->s; sc->s = gn / a1;
    sc->a1 = a1; sc->a2 = a2; sc->a3 = a3;
    sc->ceta = sc->c * sc->eta;
    sc->eta = -sc->s * sc->eta;
    sc->gamma_new = gn;
    sc->exact = (gn == 0.0);
  } else {
    sc->relres = sqrt(tot[0]) / sc->bnorm;
    sc->iter += 1;
    if (sc->relres <= sc->rtol || sc->exact) sc->status = DONE_CONV;
    else if (sc->iter >= sc->maxit) sc->status = DONE_MAXIT;
    sc->gamma_old = sc->gamma;
    sc->gamma = sc->gamma_new;
    sc->zs = 1.0 / sc->gamma_new;
  }
}

// Chebyshev helpers for P_theta (per-mode solves run on all modes at once).
// first: x = t/c scaled: dvec = a_t * tmp; x = dvec.  else x += dvec_old... see launcher.
// T: the element type of the Chebyshev vectors (float32 in a mixed-precision P^{-1}); the
// arithmetic is float64.
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_axpy(size_t len, T *__restrict__ x, T *__restrict__ dvec,
                                                   const T *__restrict__ tmp, double a_d, double a_t,
                                                   int first, const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
    const double d = first ? a_t * (double)tmp[e] : a_d * (double)dvec[e] + a_t * (double)tmp[e];
    dvec[e] = (T)d;
    x[e] = first ? (T)d : (T)((double)x[e] + d);
  }
}

// res -= (eta_j I + tau zeta_j K(a)) dvec on every time mode j.
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_resid(SP s, TileInfo ti, const double *__restrict__ ez,
                                                    T *__restrict__ res, const T *__restrict__ dvec,
                                                    const Scal *__restrict__ gate) {
  if (gate && gate->status != RUNNING) return;
  for (int t = blockIdx.x; t < ti.ntiles; t += gridDim.x) {
    int k, j, i;
    if (!tile_point(t, ti.ni, ti.nj, s.N, s.dim, k, j, i)) continue;
    const int q = (s.dim == 1) ? i : j * s.N + i;
    const T *dk = dvec + (size_t)k * s.m;
    const double av = ez[k] * (double)dk[q] + s.tau * ez[s.n + k] * Kapply<T>(s, dk, 1.0, nullptr, 0.0, j, i);
    T *r = res + (size_t)k * s.m + q;
    *r = (T)((double)*r - av);
  }
}

inline int grid_for(size_t work, int per_block) {
  size_t g = (work + per_block - 1) / per_block;
  if (g > (size_t)kRedSlots) g = kRedSlots;
  if (g < 1) g = 1;
  return (int)g;
}

// Grid of a kernel without block partial sums: one block per `per_block` items, so that no
// thread walks several items one after another (capped only by the grid-stride loops' reach)
inline int grid_all(size_t work, int per_block) {
  size_t g = (work + per_block - 1) / per_block;
  if (g > (size_t)(1 << 20)) g = 1 << 20;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_apply_YT(Ctx c, const double *x, const double *d_xscale, double *y, const double *rhs,
                           double *part, int *nblocks_out, const Scal *gate) {
  const Plan *p = c.p;
  const TileInfo ti = tiles_of(p, 1);               // spatial tiles of one level
  MarchP mp{ti.ni, ti.nj, 1, p->n};
  // runs of >= 16 levels, as many as the partial-sum slots allow
  const int maxrun = kRedSlots / ti.ntiles > 0 ? kRedSlots / ti.ntiles : 1;
  mp.nkc = std::max(1, std::min((p->n + 15) / 16, maxrun));
  mp.kr = (p->n + mp.nkc - 1) / mp.nkc;
  mp.nkc = (p->n + mp.kr - 1) / mp.kr;
  const int g = ti.ntiles * mp.nkc;
  if (g > kRedSlots) return hipErrorInvalidValue;   // more spatial tiles than partial-sum slots
  if (nblocks_out) *nblocks_out = g;
  if (rhs)
    hipLaunchKernelGGL(k_apply_YT<1>, dim3(g), block_of(p), 0, c.st, make_sp(p), mp, x, d_xscale, y, rhs, part, gate);
  else
    hipLaunchKernelGGL(k_apply_YT<0>, dim3(g), block_of(p), 0, c.st, make_sp(p), mp, x, d_xscale, y, rhs, part, gate);
  return hipGetLastError();
}

hipError_t launch_build_rhs(Ctx c, const double *f, const double *u0, double *b) {
  const Plan *p = c.p;
  TileInfo ti = tiles_of(p, p->n);
  const int g = ti.ntiles < kRedSlots ? ti.ntiles : kRedSlots;
  hipLaunchKernelGGL(k_build_rhs, dim3(g), block_of(p), 0, c.st, make_sp(p), ti, f, u0, b);
  return hipGetLastError();
}

hipError_t launch_rhs_adjoint(Ctx c, const double *lam, double *gf, double *gu0) {
  const Plan *p = c.p;
  TileInfo ti = tiles_of(p, p->n + 1);
  const int g = ti.ntiles < kRedSlots ? ti.ntiles : kRedSlots;
  hipLaunchKernelGGL(k_rhs_adjoint, dim3(g), block_of(p), 0, c.st, make_sp(p), ti, lam, gf, gu0);
  return hipGetLastError();
}

hipError_t launch_grad_faces(Ctx c, const double *u, const double *u0, const double *lam, double *gax,
                             double *gay, double *gnodal) {
  const Plan *p = c.p;
  const int N = p->N;
  const int nf = p->dim == 1 ? N + 1 : 2 * N * (N + 1);
  hipLaunchKernelGGL(k_grad_faces, dim3((nf + 255) / 256), dim3(256), 0, c.st, make_sp(p), u, u0, lam, gax, gay);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !gnodal) return e;
  const int G = N + 2;
  const int total = p->dim == 1 ? G : G * G;
  hipLaunchKernelGGL(k_grad_nodal, dim3((total + 255) / 256), dim3(256), 0, c.st, p->dim, N, gax, gay, gnodal);
  return hipGetLastError();
}

hipError_t launch_vupdate(Ctx c, const double *q, const double *v, double *vold, const Scal *gate) {
  hipLaunchKernelGGL(k_vupdate, dim3(grid_all(c.p->len, 1024)), dim3(256), 0, c.st, c.p->len, q, v, vold, gate);
  return hipGetLastError();
}

hipError_t launch_wxupdate(Ctx c, const double *z, double *wold, const double *w, double *x, const Scal *gate) {
  hipLaunchKernelGGL(k_wxupdate, dim3(grid_all(c.p->len, 1024)), dim3(256), 0, c.st, c.p->len, z, wold, w, x, gate);
  return hipGetLastError();
}

hipError_t launch_dot(Ctx c, const double *a, const double *b, double *part, int *nblocks_out, const Scal *gate) {
  const int g = grid_for(c.p->len, 1024);
  if (nblocks_out) *nblocks_out = g;
  hipLaunchKernelGGL(k_dot, dim3(g), dim3(256), 0, c.st, c.p->len, a, b, part, gate);
  return hipGetLastError();
}

hipError_t launch_scale_copy(Ctx c, const double *in, double *out, double s, int flip) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(c.p->len, 1024)), dim3(256), 0, c.st, c.p->n, c.p->m, in, out, s,
                     flip);
  return hipGetLastError();
}

hipError_t launch_zero(Ctx c, double *x, size_t len) {
  hipLaunchKernelGGL(k_zero, dim3(grid_for(len, 1024)), dim3(256), 0, c.st, len, x);
  return hipGetLastError();
}

hipError_t launch_zero_int(Ctx c, int *x, int count) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c.st, count, x);
  return hipGetLastError();
}

hipError_t launch_scalar_step(Ctx c, int stage, const double *part, int nb, const double *part2, int nb2) {
  hipLaunchKernelGGL(k_scalar_step, dim3(1), dim3(256), 0, c.st, stage, c.p->sc, part, nb, part2, nb2);
  return hipGetLastError();
}

hipError_t launch_cheb_axpy(Ctx c, void *x, void *dvec, const void *tmp, double a_d, double a_t, int first,
                            const Scal *gate, bool f32) {
  const dim3 g(grid_all(c.p->len, 1024));
  if (f32)
    hipLaunchKernelGGL(k_cheb_axpy<float>, g, dim3(256), 0, c.st, c.p->len, (float *)x, (float *)dvec,
                       (const float *)tmp, a_d, a_t, first, gate);
  else
    hipLaunchKernelGGL(k_cheb_axpy<double>, g, dim3(256), 0, c.st, c.p->len, (double *)x, (double *)dvec,
                       (const double *)tmp, a_d, a_t, first, gate);
  return hipGetLastError();
}

hipError_t launch_cheb_resid(Ctx c, void *res, const void *dvec, const Scal *gate, bool f32) {
  const Plan *p = c.p;
  TileInfo ti = tiles_of(p, p->n);
  const int g = grid_all(ti.ntiles, 1);
  if (f32)
    hipLaunchKernelGGL(k_cheb_resid<float>, dim3(g), block_of(p), 0, c.st, make_sp(p), ti, p->ez, (float *)res,
                       (const float *)dvec, gate);
  else
    hipLaunchKernelGGL(k_cheb_resid<double>, dim3(g), block_of(p), 0, c.st, make_sp(p), ti, p->ez, (double *)res,
                       (const double *)dvec, gate);
  return hipGetLastError();
}

}  // namespace smr
