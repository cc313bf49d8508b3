// C ABI of the gfx950 library (host side): validation, workspace layout, plan tables,
// the MINRES drivers and the adjoint/gradient entries.  Every step of the solve runs in
// the HIP kernels of this directory; the host only enqueues them and reads the device
// status word between chunks of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <map>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "smr_internal.h"

struct smr_plan {
  smr::Plan p;
};

namespace smr {

hipError_t lds_limit(const void *kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<const void *, int>, size_t> set;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  size_t &have = set[{kernel, dev}];
  if (bytes <= have) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) have = bytes;
  return e;
}
namespace {

thread_local std::string g_err;

smr_status fail(smr_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess)                                                                     \
      return fail(SMR_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
  } while (0)

// ---------------------------------------------------------------- event profiler
enum ProfClass { PROF_TIME = 0, PROF_DST = 1, PROF_STENCIL = 2, PROF_VEC = 3, PROF_SCALAR = 4, PROF_SPEC = 5,
                 PROF_KSLICE = 6, PROF_NCLASS = 7 };
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;                     // free events
  struct Rec {
    hipEvent_t a, b;
    int count;                                      // launches between the two events
  };
  std::vector<Rec> rec[PROF_NCLASS];
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  struct Mark {
    size_t n[PROF_NCLASS];
  };
  Mark mark() const {
    Mark k;
    for (int i = 0; i < PROF_NCLASS; ++i) k.n[i] = rec[i].size();
    return k;
  }
  void drop_back(int i) {
    pool.push_back(rec[i].back().a);
    pool.push_back(rec[i].back().b);
    rec[i].pop_back();
  }
  // drop the records made after mark k (launches that exited without work)
  void truncate(const Mark &k) {
    for (int i = 0; i < PROF_NCLASS; ++i)
      while (rec[i].size() > k.n[i]) drop_back(i);
  }
  // of class i's records after mark k keep those covering the first `keep` launches (a
  // record that straddles the limit keeps its time and counts only the launches inside)
  void keep_launches(const Mark &k, int i, long keep) {
    size_t r = k.n[i];
    long seen = 0;
    for (; r < rec[i].size() && seen < keep; ++r) {
      if (seen + rec[i][r].count > keep) rec[i][r].count = (int)(keep - seen);
      seen += rec[i][r].count;
    }
    while (rec[i].size() > r) drop_back(i);
  }
  void clear() {
    for (auto &r : rec) {
      for (auto &pr : r) {
        pool.push_back(pr.a);
        pool.push_back(pr.b);
      }
      r.clear();
    }
  }
};
Profiler g_prof;

struct ProfScope {
  int cls;
  hipStream_t st;
  int count;
  hipEvent_t a = nullptr;
  ProfScope(int c, hipStream_t s, int n = 1) : cls(c), st(s), count(n) {
    if (g_prof.on) {
      a = g_prof.get();
      if (a) hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = g_prof.get();
      if (b) {
        hipEventRecord(b, st);
        g_prof.rec[cls].push_back({a, b, count});
      } else {
        g_prof.pool.push_back(a);
      }
    }
  }
};
// Enqueue one launch on c.st, bracketed by profiler events when profiling is on.
#define LAUNCH(cls, expr)             \
  do {                                \
    ProfScope _ps((cls), c.st);       \
    HIP_TRY(expr);                    \
  } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// row stride of the sine-basis work vectors: whole 256-byte lines per 32-column tile
int ld_of(size_t m) { return (int)((m + 31) / 32 * 32); }

int hp_of(int h1) {
  int hp = 16;
  while (hp < h1) hp *= 2;
  return hp;
}

smr_status validate(const smr_desc *d) {
  if (!d) return fail(SMR_EINVAL, "desc is NULL");
  if (d->dim < 1 || d->dim > 3) return fail(SMR_EINVAL, "dim must be 1, 2 or 3 (got %d)", d->dim);
  const int maxN = d->dim == 3 ? kMaxN3 : kMaxN;
  if (d->N < 1 || d->N > maxN || !is_pow2(d->N + 1))
    return fail(SMR_EINVAL, "N + 1 must be a power of two in [2, %d] in %dD (got N = %d)", maxN + 1, d->dim, d->N);
  if (d->scheme != SMR_THETA && d->scheme != SMR_BDF2 && d->scheme != SMR_BDF3 && d->scheme != SMR_BDF4)
    return fail(SMR_EINVAL, "unknown scheme %d", d->scheme);
  const int nmin = d->scheme == SMR_THETA ? 1 : d->scheme;   // BDF-l: n >= l
  if (d->n < nmin || d->n > kMaxn) return fail(SMR_EINVAL, "n must be in [%d, %d] (got %d)", nmin, kMaxn, d->n);
  if (!(d->T > 0.0) || !std::isfinite(d->T)) return fail(SMR_EINVAL, "T must be finite and > 0");
  if (d->scheme == SMR_THETA && !(d->theta >= 0.0 && d->theta <= 1.0))
    return fail(SMR_EINVAL, "theta must lie in [0, 1] (got %g)", d->theta);
  if (d->precond != SMR_P_H && d->precond != SMR_P_THETA_CHEB && d->precond != SMR_P_NONE)
    return fail(SMR_EINVAL, "unknown preconditioner %d", d->precond);
  if (d->precond == SMR_P_THETA_CHEB && d->scheme != SMR_THETA)
    return fail(SMR_EINVAL, "P_theta is defined for the theta scheme only");
  if (d->precond == SMR_P_THETA_CHEB && (d->cheb_k < 1 || d->cheb_k > 16))
    return fail(SMR_EINVAL, "cheb_k must be in [1, 16] (got %d)", d->cheb_k);
  if (d->pprec != SMR_FP64 && d->pprec != SMR_FP32)
    return fail(SMR_EUNSUPPORTED, "pprec %d is not implemented", d->pprec);
  if (d->pprec == SMR_FP32 && d->precond == SMR_P_NONE)
    return fail(SMR_EINVAL, "float32 preconditioning needs a preconditioner (P = I has none)");
  const int known = SMR_FLAG_GENERAL_PATH | SMR_FLAG_TILE16 | SMR_FLAG_TILE32 | SMR_FLAG_TILE64 | SMR_FLAG_PINV_F64 |
                    SMR_FLAG_PINV_F32 | SMR_FLAG_PINV_F32_COL16 | SMR_FLAG_PINV_F64_COL16 | SMR_FLAG_MATVEC_LEVEL |
                    SMR_FLAG_MATVEC_TILES;
  if ((d->flags & ~known) != 0) return fail(SMR_EINVAL, "unknown flags 0x%x", d->flags);
  if ((d->flags & SMR_FLAG_MATVEC_LEVEL) && (d->flags & SMR_FLAG_MATVEC_TILES))
    return fail(SMR_EINVAL, "SMR_FLAG_MATVEC_LEVEL and SMR_FLAG_MATVEC_TILES exclude each other");
  const int pinv_flags =
      d->flags & (SMR_FLAG_PINV_F64 | SMR_FLAG_PINV_F32 | SMR_FLAG_PINV_F32_COL16 | SMR_FLAG_PINV_F64_COL16);
  if (pinv_flags & (pinv_flags - 1)) return fail(SMR_EINVAL, "at most one SMR_FLAG_PINV_* flag");
  if ((pinv_flags & (SMR_FLAG_PINV_F32 | SMR_FLAG_PINV_F32_COL16)) && d->pprec != SMR_FP32)
    return fail(SMR_EINVAL, "float32 P^-1 intermediates need pprec SMR_FP32");
  const int tile_flags = d->flags & (SMR_FLAG_TILE16 | SMR_FLAG_TILE32 | SMR_FLAG_TILE64);
  if (tile_flags & (tile_flags - 1)) return fail(SMR_EINVAL, "SMR_FLAG_TILE16/32/64 exclude each other");
  if ((d->flags & SMR_FLAG_TILE32) && !spec_cols_ok(hp_of((d->n + 1) / 2), 32))
    return fail(SMR_EUNSUPPORTED, "32-column tiles need ceil(n/2) <= 128 (got n = %d)", d->n);
  if ((d->flags & SMR_FLAG_TILE64) && !spec_cols_ok(hp_of((d->n + 1) / 2), 64, d->pprec))
    return fail(SMR_EUNSUPPORTED, "64-column tiles need ceil(n/2) <= 64, or <= 128 with SMR_FP32 (got n = %d)", d->n);
  const int forms = (d->ax_host != nullptr) + (d->a_nodal_host != nullptr);
  if (forms > 1) return fail(SMR_EINVAL, "give face values or nodal values of a, not both");
  if (d->ax_host && d->dim >= 2 && !d->ay_host) return fail(SMR_EINVAL, "dim %d face values need ay", d->dim);
  if (d->ax_host && d->dim == 3 && !d->az_host) return fail(SMR_EINVAL, "dim 3 face values need az");
  if (!d->ax_host && d->ay_host) return fail(SMR_EINVAL, "ay given without ax");
  if (d->az_host && (d->dim != 3 || !d->ax_host)) return fail(SMR_EINVAL, "az is for dim 3 face values (with ax, ay)");
  if (d->a_nodal_host && d->dim == 3) return fail(SMR_EINVAL, "3D coefficients are given as face values");
  return SMR_OK;
}

// A 2D variable-coefficient P_H solve runs in the sine basis when the per-level matvec
// supports its N (the level, N x (N + 2) float64, is held in LDS).
bool var_sine_basis(const smr_desc *d) {
  const int L = d->N + 1;
  return d->dim == 2 && (L == 32 || L == 64 || L == 128) && d->precond == SMR_P_H &&
         !(d->flags & SMR_FLAG_GENERAL_PATH) && (d->ax_host || d->a_nodal_host);
}

// The N = 127 variable-coefficient sine-basis solve can also run its per-level matvec as
// three passes over line tiles (four more level-sized intermediates in the workspace).
bool ks_split_capable(const smr_desc *d) { return var_sine_basis(d) && d->N + 1 == 128; }

// interior points and face values per axis array: m = N^dim; faces along one axis (N+1) N^(dim-1)
size_t m_of(int dim, int N) { return dim == 1 ? (size_t)N : dim == 2 ? (size_t)N * N : (size_t)N * N * N; }
size_t faces_of(int dim, int N) { return m_of(dim, N) / N * (N + 1); }

struct Layout {
  size_t ax, ay, az, tmu, tmu_lap, tcoef, ez, So, SoT, Se, SeT, Sof, SoTf, Sef, SeTf, zf, tw, gface, part, sc, vec0;
  int nvec;
  size_t total;
};

Layout layout_of(const smr_desc *d) {
  const int N = d->N, n = d->n, dim = d->dim;
  const size_t m = m_of(dim, N);
  const size_t len = (size_t)ld_of(m) * n;   // every work vector holds n rows of ld
  const int hp = hp_of((n + 1) / 2);
  const int L = N + 1;
  Layout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align256(off + (bytes ? bytes : 8));
    return at;
  };
  l.ax = take(sizeof(double) * faces_of(dim, N));
  l.ay = take(sizeof(double) * (dim == 1 ? 1 : faces_of(dim, N)));
  l.az = take(sizeof(double) * (dim == 3 ? faces_of(dim, N) : 1));
  l.tmu = take(sizeof(double) * m);
  l.tmu_lap = take(sizeof(double) * m);
  l.tcoef = take(sizeof(double) * 4 * (size_t)n);
  l.ez = take(sizeof(double) * 2 * (size_t)n);
  l.So = take(sizeof(double) * hp * hp);
  l.SoT = take(sizeof(double) * hp * hp);
  l.Se = take(sizeof(double) * hp * hp);
  l.SeT = take(sizeof(double) * hp * hp);
  const bool f32 = d->pprec == SMR_FP32;
  l.Sof = take(f32 ? sizeof(float) * hp * hp : 0);
  l.SoTf = take(f32 ? sizeof(float) * hp * hp : 0);
  l.Sef = take(f32 ? sizeof(float) * hp * hp : 0);
  l.SeTf = take(f32 ? sizeof(float) * hp * hp : 0);
  l.zf = take(f32 ? 3 * align256(sizeof(float) * len) : 0);
  l.tw = take(sizeof(double) * 2 * (size_t)L);
  l.gface = take(sizeof(double) * 2 * (size_t)(N + 1) * (N + 1));
  l.part = take(sizeof(double) * spec_part_doubles((int)m));
  l.sc = take(2 * sizeof(Scal));
  // V0 V1 Z0 Z1 W0 W1 Q T1 T2 G (+ T3 T4 for the Chebyshev inner solve, + QX for the
  // variable-coefficient sine-basis solve)
  l.nvec = 10 + (d->precond == SMR_P_THETA_CHEB ? 2 : 0) + (var_sine_basis(d) ? 1 : 0) + (ks_split_capable(d) ? 4 : 0);
  l.vec0 = off;
  off += (size_t)l.nvec * align256(sizeof(double) * len);
  l.total = off;
  return l;
}

// sin(k pi / q) for integer k, reduced exactly before the long-double evaluation
long double sinpi_ratio(long long k, long long q) {
  long long r = k % (2 * q);
  if (r < 0) r += 2 * q;
  return sinl((long double)r * 3.14159265358979323846264338327950288L / (long double)q);
}
long double cospi_ratio(long long k, long long q) {
  long long r = k % (2 * q);
  if (r < 0) r += 2 * q;
  return cosl((long double)r * 3.14159265358979323846264338327950288L / (long double)q);
}

// The averaged Toeplitz Kbar of Sec. 3.1.1: d = mean of h^2 diag(K), c_axis = mean of the
// interior face values along each axis (long double sums, fixed order).
void mean_faces(const Plan &p, const std::vector<double> &ax, const std::vector<double> &ay,
                const std::vector<double> &az, double &d, double &cx, double &cy, double &cz) {
  const long long N = p.N;
  long double sd = 0, sx = 0, sy = 0, sz = 0;
  cx = cy = cz = 0.0;
  if (p.dim == 1) {
    for (int i = 0; i < N; ++i) sd += (long double)ax[i] + ax[i + 1];
    for (int i = 1; i < N; ++i) sx += ax[i];
    d = (double)(sd / N);
    if (N > 1) cx = (double)(sx / (N - 1));
    return;
  }
  // planes (one in 2D): ax[k][j][i] (N+1 per row), ay[k][j][i] (N+1 rows per plane), az[k][j][i]
  const long long P = p.dim == 3 ? N : 1;
  for (long long k = 0; k < P; ++k)
    for (long long j = 0; j < N; ++j)
      for (long long i = 0; i < N; ++i) {
        const size_t xa = (size_t)((k * N + j) * (N + 1) + i), ya = (size_t)((k * (N + 1) + j) * N + i);
        sd += (long double)ax[xa] + ax[xa + 1] + ay[ya] + ay[ya + N];
        if (p.dim == 3) sd += (long double)az[(size_t)((k * N + j) * N + i)] + az[(size_t)(((k + 1) * N + j) * N + i)];
        if (i >= 1) sx += ax[xa];
        if (j >= 1) sy += ay[ya];
        if (p.dim == 3 && k >= 1) sz += az[(size_t)((k * N + j) * N + i)];
      }
  const long double cnt = (long double)P * N * N, inner = (long double)P * N * (N - 1);
  d = (double)(sd / cnt);
  if (N > 1) {
    cx = (double)(sx / inner);
    cy = (double)(sy / inner);
    if (p.dim == 3) cz = (double)(sz / inner);
  }
}

// compute units of the current device (256 on MI355X)
int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

// Times the physical-basis P^{-1} variants of a float32 plan and sets p.pinv_var (defined below).
smr_status pinv_tune(Plan &p, hipStream_t s);
smr_status kslice_tune(Plan &p, hipStream_t s);

// P_H / Phat (any a the sine-basis path takes), and P_theta of a constant a (its per-mode
// blocks are diagonal in the spatial sine basis)
bool use_spectral(const Plan &p) {
  if (p.flags & SMR_FLAG_GENERAL_PATH) return false;
  if (p.precond == SMR_P_H) return p.const_coef || p.QX != nullptr;
  return p.precond == SMR_P_THETA_CHEB && p.const_coef;
}

}  // namespace
}  // namespace smr

using namespace smr;

extern "C" {

const char *smr_version(void) { return "smr 0.1 (gfx950, fp64)"; }

const char *smr_last_error(void) { return g_err.c_str(); }

smr_status smr_workspace_size(const smr_desc *desc, size_t *bytes) {
  smr_status st = validate(desc);
  if (st != SMR_OK) return st;
  if (!bytes) return fail(SMR_EINVAL, "bytes is NULL");
  *bytes = layout_of(desc).total;
  return SMR_OK;
}

smr_status smr_setup(const smr_desc *d, void *d_ws, size_t ws_bytes, void *stream, smr_plan **out) {
  smr_status st = validate(d);
  if (st != SMR_OK) return st;
  if (!out) return fail(SMR_EINVAL, "out is NULL");
  *out = nullptr;
  const Layout lay = layout_of(d);
  if (!d_ws) return fail(SMR_EWORKSPACE, "workspace is NULL");
  if (((uintptr_t)d_ws & 255) != 0) return fail(SMR_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < lay.total) return fail(SMR_EWORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, lay.total);
  hipStream_t s = (hipStream_t)stream;

  smr_plan *pl = new (std::nothrow) smr_plan();
  if (!pl) return fail(SMR_EINVAL, "out of host memory");
  Plan &p = pl->p;
  p.dim = d->dim;
  p.N = d->N;
  p.n = d->n;
  p.m = (int)m_of(d->dim, d->N);
  p.len = (size_t)p.m * p.n;
  p.ld = ld_of((size_t)p.m);
  p.vlen = (size_t)p.ld * p.n;
  p.scheme = d->scheme;
  p.precond = d->precond;
  p.pprec = d->pprec;
  p.cheb_k = d->cheb_k;
  p.flags = d->flags;
  p.T = d->T;
  p.tau = d->T / d->n;
  p.theta = d->scheme == SMR_THETA ? d->theta : 1.0;
  p.taps = scheme_coefs(p.scheme, p.theta, p.tcf, p.kbf);
  p.L = d->N + 1;
  p.logL = ilog2(p.L);
  p.h = 1.0 / p.L;
  p.h2inv = (double)p.L * (double)p.L;
  p.h1 = (d->n + 1) / 2;
  p.h2 = d->n / 2;
  p.hp = hp_of(p.h1);
  p.spec_c = (d->flags & SMR_FLAG_TILE16)   ? 16
             : (d->flags & SMR_FLAG_TILE32) ? 32
             : (d->flags & SMR_FLAG_TILE64) ? 64
                                            : spec_cols_default(p.hp);
  p.ws_bytes = ws_bytes;

  const int N = p.N, n = p.n, m = p.m, dim = p.dim;
  // ---- face values
  const size_t nax = faces_of(dim, N);
  const size_t nay = dim == 1 ? 0 : faces_of(dim, N);
  const size_t naz = dim == 3 ? faces_of(dim, N) : 0;
  std::vector<double> ax(nax, 1.0), ay(std::max<size_t>(nay, 1), 1.0), az(std::max<size_t>(naz, 1), 1.0);
  if (d->ax_host) {
    std::copy(d->ax_host, d->ax_host + nax, ax.begin());
    if (dim >= 2) std::copy(d->ay_host, d->ay_host + nay, ay.begin());
    if (dim == 3) std::copy(d->az_host, d->az_host + naz, az.begin());
  } else if (d->a_nodal_host) {
    const double *a = d->a_nodal_host;
    const int G = N + 2;
    if (dim == 1) {
      for (int i = 0; i <= N; ++i) ax[i] = 0.5 * (a[i] + a[i + 1]);
    } else {
      for (int j = 0; j < N; ++j)
        for (int i = 0; i <= N; ++i) ax[j * (N + 1) + i] = 0.5 * (a[(j + 1) * G + i] + a[(j + 1) * G + i + 1]);
      for (int j = 0; j <= N; ++j)
        for (int i = 0; i < N; ++i) ay[j * N + i] = 0.5 * (a[j * G + i + 1] + a[(j + 1) * G + i + 1]);
    }
  }
  double amin = ax[0], amax = ax[0];
  for (size_t i = 0; i < nax; ++i) {
    if (!(ax[i] > 0.0) || !std::isfinite(ax[i])) {
      delete pl;
      return fail(SMR_EINVAL, "face value ax[%zu] = %g is not finite and positive", i, ax[i]);
    }
    amin = std::min(amin, ax[i]);
    amax = std::max(amax, ax[i]);
  }
  for (size_t i = 0; i < nay; ++i) {
    if (!(ay[i] > 0.0) || !std::isfinite(ay[i])) {
      delete pl;
      return fail(SMR_EINVAL, "face value ay[%zu] = %g is not finite and positive", i, ay[i]);
    }
    amin = std::min(amin, ay[i]);
    amax = std::max(amax, ay[i]);
  }
  for (size_t i = 0; i < naz; ++i) {
    if (!(az[i] > 0.0) || !std::isfinite(az[i])) {
      delete pl;
      return fail(SMR_EINVAL, "face value az[%zu] = %g is not finite and positive", i, az[i]);
    }
    amin = std::min(amin, az[i]);
    amax = std::max(amax, az[i]);
  }
  p.a_min = amin;
  p.a_max = amax;
  p.const_coef = (amin == amax);
  p.abar = 0.5 * (amin + amax);
  p.cheb_lo = std::min(1.0, amin / p.abar);
  p.cheb_hi = std::max(1.0, amax / p.abar);
  mean_faces(p, ax, ay, az, p.kbar_d, p.kbar_cx, p.kbar_cy, p.kbar_cz);

  // ---- spatial eigenvalues (sine-basis order, x fastest), tau included
  std::vector<double> s2(N);
  for (int k = 0; k < N; ++k) {
    const long double sv = sinpi_ratio(k + 1, 2LL * p.L);
    s2[k] = (double)(sv * sv);
  }
  std::vector<double> tmu(m), tmul(m);
  const double base = p.kbar_d - 2.0 * (p.kbar_cx + p.kbar_cy + p.kbar_cz);   // cy = 0 in 1D, cz = 0 below 3D
  for (int q = 0; q < m; ++q) {
    const int kx = q % N, ly = (q / N) % N, lz = q / (N * N);
    double mu = base + 4.0 * p.kbar_cx * s2[kx];
    double ml = 4.0 * s2[kx];
    if (dim >= 2) {
      mu += 4.0 * p.kbar_cy * s2[ly];
      ml += 4.0 * s2[ly];
    }
    if (dim == 3) {
      mu += 4.0 * p.kbar_cz * s2[lz];
      ml += 4.0 * s2[lz];
    }
    tmu[q] = p.tau * (mu * p.h2inv);
    tmul[q] = p.tau * (ml * p.h2inv);
  }
  // ---- time-mode coefficients: sigma_j = |(A + t B) + i (C + t D)| and eta_j, zeta_j
  std::vector<double> tcoef(4 * (size_t)n), ez(2 * (size_t)n);
  const double th = p.theta;
  for (int t = 0; t < n; ++t) {
    const long double sp = sinpi_ratio(t + 1, n + 1);           // sin(phi)
    const long double cp = cospi_ratio(t + 1, n + 1);           // cos(phi)
    const long double sh = sinpi_ratio(t + 1, 2LL * (n + 1));   // sin(phi/2)
    const long double s2h = sh * sh;
    if (p.precond == SMR_P_THETA_CHEB) {
      // P_theta of a constant a: eta_j + tau zeta_j mu (used by the sine-basis path only)
      tcoef[4 * t + 0] = (double)(2.0L * sh);
      tcoef[4 * t + 1] = (double)sqrtl(th * th + (1.0L - th) * (1.0L - th) + 2.0L * th * (1.0L - th) * cp);
      tcoef[4 * t + 2] = 0.0;
      tcoef[4 * t + 3] = 0.0;
    } else if (p.scheme == SMR_THETA) {
      tcoef[4 * t + 0] = (double)(2.0L * s2h);
      tcoef[4 * t + 1] = (double)(th + (1.0L - th) * cp);
      tcoef[4 * t + 2] = (double)(-sp);
      tcoef[4 * t + 3] = (double)((1.0L - th) * sp);
    } else if (p.scheme == SMR_BDF2) {
      tcoef[4 * t + 0] = (double)(4.0L * s2h * s2h);
      tcoef[4 * t + 1] = 1.0;
      tcoef[4 * t + 2] = (double)(-sp * (2.0L - cp));
      tcoef[4 * t + 3] = 0.0;
    } else {
      // ghat(phi) at tau mu = (alpha_0 + tau mu) + sum_{k >= 1} alpha_k e^{i k phi}; since the
      // alpha_k sum to zero its real part is tau mu - 2 sum_k alpha_k sin^2(k phi / 2)
      long double re = 0.0L, im = 0.0L;
      for (int k = 1; k < p.taps; ++k) {
        const long double hk = sinpi_ratio((long long)k * (t + 1), 2LL * (n + 1));
        re += -2.0L * p.tcf[k] * hk * hk;
        im += p.tcf[k] * sinpi_ratio((long long)k * (t + 1), n + 1);
      }
      tcoef[4 * t + 0] = (double)re;
      tcoef[4 * t + 1] = 1.0;
      tcoef[4 * t + 2] = (double)im;
      tcoef[4 * t + 3] = 0.0;
    }
    ez[t] = (double)(2.0L * sh);
    ez[n + t] = (double)sqrtl(th * th + (1.0L - th) * (1.0L - th) + 2.0L * th * (1.0L - th) * cp);
  }
  // smallest eigenvalue of P: a lower bound ||r||_2 >= sqrt(min sigma) ||r||_{P^-1}
  {
    double smin = INFINITY;
    for (int t = 0; t < n; ++t) {
      const double A = tcoef[4 * t], B = tcoef[4 * t + 1], Cc = tcoef[4 * t + 2], Dd = tcoef[4 * t + 3];
      for (int q = 0; q < m; ++q) {
        const double re = A + tmu[q] * B, im = Cc + tmu[q] * Dd;
        smin = std::min(smin, re * re + im * im);
      }
    }
    p.sqsigmin = std::sqrt(std::sqrt(smin));
  }
  // ---- folded time sine blocks in MFMA fragment order
  const int hp = p.hp, KS = hp / 4;
  const long double nrm = sqrtl(2.0L / (n + 1));
  auto Sval = [&](long long i1, long long j1) { return (double)(nrm * sinpi_ratio(i1 * j1, n + 1)); };
  auto So = [&](int pp, int qq) { return (pp < p.h1 && qq < p.h1) ? Sval(2LL * pp + 1, qq + 1) : 0.0; };
  auto Se = [&](int pp, int qq) { return (pp < p.h2 && qq < p.h2) ? Sval(2LL * pp + 2, qq + 1) : 0.0; };
  std::vector<double> fo(hp * hp), foT(hp * hp), fe(hp * hp), feT(hp * hp);
  for (int r = 0; r < hp / 16; ++r)
    for (int kk = 0; kk < KS; ++kk)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = 16 * r + (lane & 15), k = 4 * kk + (lane >> 4);
        // fragments of k-steps 2q and 2q+1 adjacent per lane: one 16-byte load fetches both
        const size_t at = (((size_t)r * (KS / 2) + kk / 2) * 64 + lane) * 2 + (kk & 1);
        fo[at] = So(i, k);
        foT[at] = So(k, i);
        fe[at] = Se(i, k);
        feT[at] = Se(k, i);
      }
  std::vector<float> fof, foTf, fef, feTf;
  if (p.pprec == SMR_FP32) {
    fof.assign(fo.begin(), fo.end());
    foTf.assign(foT.begin(), foT.end());
    fef.assign(fe.begin(), fe.end());
    feTf.assign(feT.begin(), feT.end());
  }
  // ---- FFT twiddles exp(-2 pi i t / (2L)), t < L
  std::vector<double> tw(2 * (size_t)p.L);
  for (int t = 0; t < p.L; ++t) {
    tw[2 * t] = (double)cospi_ratio(t, p.L);
    tw[2 * t + 1] = (double)(-sinpi_ratio(t, p.L));
  }

  char *base_ptr = (char *)d_ws;
  p.ax = (double *)(base_ptr + lay.ax);
  p.ay = (double *)(base_ptr + lay.ay);
  p.az = (double *)(base_ptr + lay.az);
  p.tmu = (double *)(base_ptr + lay.tmu);
  p.tmu_lap = (double *)(base_ptr + lay.tmu_lap);
  p.tcoef = (double *)(base_ptr + lay.tcoef);
  p.ez = (double *)(base_ptr + lay.ez);
  p.So = (double *)(base_ptr + lay.So);
  p.SoT = (double *)(base_ptr + lay.SoT);
  p.Se = (double *)(base_ptr + lay.Se);
  p.SeT = (double *)(base_ptr + lay.SeT);
  p.tw = (double *)(base_ptr + lay.tw);
  p.Sof = (float *)(base_ptr + lay.Sof);
  p.SoTf = (float *)(base_ptr + lay.SoTf);
  p.Sef = (float *)(base_ptr + lay.Sef);
  p.SeTf = (float *)(base_ptr + lay.SeTf);
  for (int i = 0; i < 3; ++i)
    p.ZF[i] = (float *)(base_ptr + lay.zf + (size_t)i * align256(sizeof(float) * p.vlen));
  p.gface = (double *)(base_ptr + lay.gface);
  p.part = (double *)(base_ptr + lay.part);
  p.sc = (Scal *)(base_ptr + lay.sc);
  const size_t vstride = align256(sizeof(double) * p.vlen);
  double *vec[16] = {};
  for (int i = 0; i < lay.nvec; ++i) vec[i] = (double *)(base_ptr + lay.vec0 + (size_t)i * vstride);
  p.V[0] = vec[0]; p.V[1] = vec[1];
  p.Z[0] = vec[2]; p.Z[1] = vec[3];
  p.W[0] = vec[4]; p.W[1] = vec[5];
  p.Q = vec[6]; p.T1 = vec[7]; p.T2 = vec[8]; p.G = vec[9];
  const bool cheb = p.precond == SMR_P_THETA_CHEB;
  p.T3 = cheb ? vec[10] : nullptr;
  p.T4 = cheb ? vec[11] : nullptr;
  p.QX = var_sine_basis(d) ? vec[lay.nvec - 1] : nullptr;
  for (int i = 0; i < 4; ++i) p.Y[i] = ks_split_capable(d) ? vec[lay.nvec - 5 + i] : nullptr;
  p.ks_split = false;

  auto up = [&](void *dst, const void *src, size_t bytes) { return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s); };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(p.ax, ax.data(), nax * sizeof(double));
  if (e == hipSuccess && nay) e = up(p.ay, ay.data(), nay * sizeof(double));
  if (e == hipSuccess && naz) e = up(p.az, az.data(), naz * sizeof(double));
  if (e == hipSuccess) e = up(p.tmu, tmu.data(), m * sizeof(double));
  if (e == hipSuccess) e = up(p.tmu_lap, tmul.data(), m * sizeof(double));
  if (e == hipSuccess) e = up(p.tcoef, tcoef.data(), tcoef.size() * sizeof(double));
  if (e == hipSuccess) e = up(p.ez, ez.data(), ez.size() * sizeof(double));
  if (e == hipSuccess) e = up(p.So, fo.data(), fo.size() * sizeof(double));
  if (e == hipSuccess) e = up(p.SoT, foT.data(), foT.size() * sizeof(double));
  if (e == hipSuccess) e = up(p.Se, fe.data(), fe.size() * sizeof(double));
  if (e == hipSuccess) e = up(p.SeT, feT.data(), feT.size() * sizeof(double));
  if (e == hipSuccess) e = up(p.tw, tw.data(), tw.size() * sizeof(double));
  if (e == hipSuccess && p.pprec == SMR_FP32) {
    e = up(p.Sof, fof.data(), fof.size() * sizeof(float));
    if (e == hipSuccess) e = up(p.SoTf, foTf.data(), foTf.size() * sizeof(float));
    if (e == hipSuccess) e = up(p.Sef, fef.data(), fef.size() * sizeof(float));
    if (e == hipSuccess) e = up(p.SeTf, feTf.data(), feTf.size() * sizeof(float));
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete pl;
    return fail(SMR_EDEVICE, "setup upload failed: %s", hipGetErrorString(e));
  }
  // the N = 127 per-level matvec: one level per block or three tiled passes, forced by a flag,
  // else timed (before the fused kernel's width, whose variable-coefficient partial count
  // depends on it)
  if (p.Y[0] && use_spectral(p)) {
    if (p.flags & SMR_FLAG_MATVEC_TILES) p.ks_split = true;
    else if (!(p.flags & SMR_FLAG_MATVEC_LEVEL)) {
      const smr_status ts = kslice_tune(p, s);
      if (ts != SMR_OK) {
        delete pl;
        return ts;
      }
    }
  }
  if (use_spectral(p) && !(p.flags & (SMR_FLAG_TILE16 | SMR_FLAG_TILE32 | SMR_FLAG_TILE64))) {
    e = spec_tune(&p, s);
    if (e != hipSuccess) {
      delete pl;
      return fail(SMR_EDEVICE, "tile-width timing failed: %s", hipGetErrorString(e));
    }
  }
  // the physical-basis P^{-1} variant: forced by a flag, else timed
  p.pinv_var = -1;
  if (!use_spectral(p) && p.precond != SMR_P_NONE) {
    const bool tiles = dst_tile_supported(&p);
    if (p.flags & SMR_FLAG_PINV_F64) p.pinv_var = 0;
    else if (p.flags & SMR_FLAG_PINV_F32) p.pinv_var = 1;
    else if (p.flags & SMR_FLAG_PINV_F32_COL16) p.pinv_var = tiles ? 2 : 1;
    else if (p.flags & SMR_FLAG_PINV_F64_COL16) p.pinv_var = tiles ? 3 : 0;
    else {
      const smr_status ts = pinv_tune(p, s);
      if (ts != SMR_OK) {
        delete pl;
        return ts;
      }
    }
  }
  *out = pl;
  return SMR_OK;
}

smr_status smr_destroy(smr_plan *plan) {
  if (plan) {
    const Plan &p = plan->p;
    if (p.steady6) hipGraphExecDestroy(p.steady6);
    if (p.snap) hipHostFree(p.snap);
    for (hipEvent_t e : p.snap_ev)
      if (e) hipEventDestroy(e);
    if (p.cap) hipStreamDestroy(p.cap);
  }
  delete plan;
  return SMR_OK;
}

}  // extern "C"

namespace smr {
namespace {

smr_status check_plan(const smr_plan *pl) {
  if (!pl) return fail(SMR_EINVAL, "plan is NULL");
  return SMR_OK;
}

// Intermediate vectors of one P^{-1} application (n*m doubles each; t3, t4 for P_theta only).
struct PinvBufs {
  double *t1, *t2, *t3, *t4;
};
PinvBufs plan_bufs(const Plan &p) { return PinvBufs{p.T1, p.T2, p.T3, p.T4}; }

// z = P^{-1} v; gamma^2 partials (Parseval or an explicit dot) into part2, count in *nb2.
// f32 (the solves of an SMR_FP32 plan): the time transforms on the float32 matrix cores and,
// per the plan's tuned variant, every intermediate vector of P^{-1} (spatial passes,
// Chebyshev steps) stored in float32 in the first half of the float64 buffers; v and z, the
// transforms' arithmetic and the Chebyshev recurrence coefficients stay float64.
smr_status apply_pinv(const Plan &p, hipStream_t s, const double *v, double *z, double *part2, int *nb2,
                      const Scal *gate, bool f32, const PinvBufs &tb) {
  Ctx c{&p, s};
  if (p.precond == SMR_P_NONE) {
    HIP_TRY(hipMemcpyAsync(z, v, p.len * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (part2) LAUNCH(PROF_VEC, launch_dot(c, z, v, part2, nb2, gate));
    return SMR_OK;
  }
  // the plan's tuned variant: float32 intermediates (float32 solves only), 16-line column tiles
  const bool w = f32 && (p.pinv_var == 1 || p.pinv_var == 2);
  const bool c16 = p.pinv_var == 2 || p.pinv_var == 3;
  if (p.precond == SMR_P_H) {
    LAUNCH(PROF_DST, launch_dst_v(c, 0, v, false, tb.t1, w, p.n, 0, gate, 0, 0, c16));
    for (int ax = 1; ax < p.dim; ++ax)
      LAUNCH(PROF_DST, launch_dst_v(c, ax, tb.t1, w, tb.t1, w, p.n, 0, gate, 0, 0, c16));
    if (w) LAUNCH(PROF_TIME, launch_time_v(c, tb.t1, true, tb.t2, true, 1, part2, nb2, gate));
    else LAUNCH(PROF_TIME, launch_time(c, tb.t1, tb.t2, 1, part2, nb2, gate, f32));
    for (int ax = p.dim - 1; ax >= 1; --ax)
      LAUNCH(PROF_DST, launch_dst_v(c, ax, tb.t2, w, tb.t2, w, p.n, 0, gate, 0, 0, c16));
    LAUNCH(PROF_DST, launch_dst_v(c, 0, tb.t2, w, z, false, p.n, 0, gate, 0, 0, c16));
    return SMR_OK;
  }
  // P_theta with k-step Chebyshev per time mode: res = T1, x = T2, dvec = T3, tmp = T4
  if (w) LAUNCH(PROF_TIME, launch_time_v(c, v, false, tb.t1, true, 0, nullptr, nullptr, gate));
  else LAUNCH(PROF_TIME, launch_time(c, v, tb.t1, 0, nullptr, nullptr, gate, f32));
  const double cc = 0.5 * (p.cheb_hi + p.cheb_lo), dd = 0.5 * (p.cheb_hi - p.cheb_lo);
  // one Chebyshev step: the inner preconditioner applied to the residual (the spatial
  // transform along every axis, the last pass dividing by the diagonal, then back) into tmp,
  // then dvec = a_t tmp (first) or a_d dvec + a_t tmp and x = dvec (first) or x + dvec.  2D
  // with N + 1 = 256: the two middle column passes run as one (divide in the tile, transform
  // again) and the last row pass applies the update in place of storing tmp.
  auto cheb_step = [&](double a_d, double a_t, int first) -> smr_status {
    const double *in = tb.t1;
    double *out = tb.t4;
    const int last = p.dim - 1;
    if (p.dim == 2 && p.L == 256 && dst_tile_supported(&p)) {
      LAUNCH(PROF_DST, launch_dst_v(c, 0, in, w, out, w, p.n, 0, gate, 0, 0, c16));
      LAUNCH(PROF_DST, launch_dst_v(c, 1, out, w, out, w, p.n, 2, gate, 0, 0, c16));
      LAUNCH(PROF_DST, launch_dst_cheb_axpy(c, out, tb.t2, tb.t3, w, a_d, a_t, first, gate));
      return SMR_OK;
    }
    LAUNCH(PROF_DST, launch_dst_v(c, 0, in, w, out, w, p.n, last == 0 ? 1 : 0, gate, 0, 0, c16));
    for (int ax = 1; ax <= last; ++ax)
      LAUNCH(PROF_DST, launch_dst_v(c, ax, out, w, out, w, p.n, ax == last ? 1 : 0, gate, 0, 0, c16));
    for (int ax = last; ax >= 0; --ax) LAUNCH(PROF_DST, launch_dst_v(c, ax, out, w, out, w, p.n, 0, gate, 0, 0, c16));
    LAUNCH(PROF_VEC, launch_cheb_axpy(c, tb.t2, tb.t3, tb.t4, a_d, a_t, first, gate, w));
    return SMR_OK;
  };
  smr_status st = cheb_step(0.0, 1.0 / cc, 1);
  if (st != SMR_OK) return st;
  if (dd > 0.0) {
    const double s1 = cc / dd;
    double rho = 1.0 / s1;
    for (int i = 1; i < p.cheb_k; ++i) {
      LAUNCH(PROF_STENCIL, launch_cheb_resid(c, tb.t1, tb.t3, gate, w));
      const double rn = 1.0 / (2.0 * s1 - rho);
      st = cheb_step(rn * rho, 2.0 * rn / dd, 0);
      if (st != SMR_OK) return st;
      rho = rn;
    }
  }
  if (w) LAUNCH(PROF_TIME, launch_time_v(c, tb.t2, true, z, false, 0, nullptr, nullptr, gate));
  else LAUNCH(PROF_TIME, launch_time(c, tb.t2, z, 0, nullptr, nullptr, gate, f32));
  if (part2) LAUNCH(PROF_VEC, launch_dot(c, z, v, part2, nb2, gate));
  return SMR_OK;
}

// The physical-basis P^{-1} variant: the spatial transform's column passes with 8- or 16-line
// tiles, and for a float32 plan float64 or float32 intermediate vectors (float32 only inside
// the time transform's GEMMs, or everywhere).  Which is fastest depends on the shape (the
// spatial passes are bound by memory-instruction issue as much as by bytes), so a few
// applications of each are timed on the plan's workspace and the fastest kept (variant 0
// unless another is 3% faster).
// Per-level matvec of an N = 127 variable-coefficient plan: time a few steady launches of each
// form on the plan's workspace (a benign running scalar state in slot 0, which a launch with
// j = 7 reads; the residual chain runs or not alike in both) and keep the tiled passes unless
// the level kernel is 3% faster.  Cached per device and shape.
smr_status kslice_tune(Plan &p, hipStream_t s) {
  const std::vector<long> key{TUNE_KSLICE, p.dim, p.N, p.n, p.scheme, p.pprec};
  int cached = 0;
  if (tune_get(key, &cached)) {
    p.ks_split = cached != 0;
    return SMR_OK;
  }
  p.ks_split = false;
  hipError_t e = spec_tune_state(&p, s, spec_desc(&p, p.T2, p.T1, p.spec_c));
  float ms[2] = {0.0f, 0.0f};
  for (int v = 0; v < 2 && e == hipSuccess; ++v) {
    p.ks_split = v == 1;
    Ctx c{&p, s};
    e = tune_time(s, 3, [&]() { return launch_kslice(c, 1, 7, p.T2, p.T1); }, &ms[v]);
  }
  if (e != hipSuccess) return fail(SMR_EDEVICE, "timing the per-level matvec failed: %s", hipGetErrorString(e));
  p.ks_split = !(ms[0] < 0.97f * ms[1]);
  tune_put(key, p.ks_split ? 1 : 0);
  return SMR_OK;
}

smr_status pinv_tune(Plan &p, hipStream_t s) {
  std::vector<int> cand{0};
  if (dst_tile_supported(&p)) cand.push_back(3);
  if (p.pprec == SMR_FP32) {
    cand.push_back(1);
    if (dst_tile_supported(&p)) cand.push_back(2);
  }
  if (cand.size() == 1) {
    p.pinv_var = 0;
    return SMR_OK;
  }
  const std::vector<long> key{TUNE_PINV, p.dim, p.N, p.n, p.precond, p.cheb_k, p.scheme, p.pprec};
  int cached = 0;
  if (tune_get(key, &cached)) {
    p.pinv_var = cached;
    return SMR_OK;
  }
  HIP_TRY(hipMemsetAsync(p.V[0], 0, p.len * sizeof(double), s));
  float best = 1e30f;
  int arg = 0;
  for (int v : cand) {
    p.pinv_var = v;
    float ms = 0.0f;
    const hipError_t e = tune_time(s, 3, [&]() -> hipError_t {
      int nb2 = 0;
      const smr_status st =
          apply_pinv(p, s, p.V[0], p.Z[0], p.part + 2 * kRedSlots, &nb2, nullptr, p.pprec == SMR_FP32, plan_bufs(p));
      return st == SMR_OK ? hipSuccess : hipErrorLaunchFailure;
    }, &ms);
    if (e != hipSuccess) return fail(SMR_EDEVICE, "timing the P^-1 variants failed: %s", hipGetErrorString(e));
    if (v == 0 || ms < 0.97f * best) {
      best = v == 0 ? ms : std::min(best, ms);
      arg = v;
    }
  }
  p.pinv_var = arg;
  tune_put(key, arg);
  return SMR_OK;
}

// spatial sine transform of every time slice (involutory: the same call transforms back);
// slice strides of in and out (m for physical vectors, ld for sine-basis ones)
smr_status spatial_dst(const Plan &p, hipStream_t s, const double *in, double *out, long in_ld, long out_ld) {
  Ctx c{&p, s};
  if (kslice_supported(&p) && in != out) {   // the whole level in LDS: one pass
    LAUNCH(PROF_DST, launch_dst2d(c, in, out, in_ld, out_ld));
    return SMR_OK;
  }
  LAUNCH(PROF_DST, launch_dst(c, 0, in, out, p.n, 0, nullptr, in_ld, out_ld));
  for (int ax = 1; ax < p.dim; ++ax) LAUNCH(PROF_DST, launch_dst(c, ax, out, out, p.n, 0, nullptr, out_ld, out_ld));
  return SMR_OK;
}
smr_status to_sine_basis(const Plan &p, hipStream_t s, const double *in, double *out) {
  return spatial_dst(p, s, in, out, p.m, p.ld);
}
smr_status from_sine_basis(const Plan &p, hipStream_t s, const double *in, double *out) {
  return spatial_dst(p, s, in, out, p.ld, p.m);
}

smr_status finish_info(const Scal &h, int maxit, smr_info *info, int tile_cols = 0) {
  smr_status res = SMR_OK;
  switch (h.status) {
    case DONE_CONV: res = SMR_OK; break;
    case DONE_NOTSPD: res = fail(SMR_ENOTSPD, "preconditioner not SPD on the residual (gamma^2 <= 0 or not finite)"); break;
    case DONE_BREAKDOWN: res = fail(SMR_EBREAKDOWN, "MINRES breakdown (alpha1 = 0)"); break;
    default: res = fail(SMR_ENOTCONV, "maxit = %d reached, relres = %g", maxit, h.relres); break;
  }
  if (info) {
    info->iters = h.iter;
    info->status = res;
    info->relres_true = h.bnorm == 0.0 ? 0.0 : h.relres;
    info->relres_prec = h.gamma1 > 0.0 ? std::fabs(h.eta) / h.gamma1 : 0.0;
    info->res_evals = h.nres;
    info->tile_cols = tile_cols;
  }
  return res;
}

// Pinned host status snapshots of a plan (two, used alternately) and their events.
smr_status ensure_snapshots(const Plan &p) {
  if (!p.snap) HIP_TRY(hipHostMalloc((void **)&p.snap, 2 * sizeof(Scal), hipHostMallocDefault));
  for (hipEvent_t &e : p.snap_ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return SMR_OK;
}

// Graphs are captured on a stream of their own (the caller's stream may be the legacy default
// stream, which cannot be captured); default priority, never used to run work.  A plan owns
// the one its single solves capture on (made on first use, destroyed with the plan).
hipStream_t plan_capture_stream(const Plan &p) {
  if (!p.cap && hipStreamCreateWithFlags(&p.cap, hipStreamNonBlocking) != hipSuccess) p.cap = nullptr;
  return p.cap;
}

// Six consecutive steady launches j = 6..11 of the sine-basis solve (with the per-level
// matvec for a variable coefficient), captured once per plan.  Their arguments depend on j
// only through j mod 6 (buffer rotation, launch parity) and j >= 3, so the same graph runs
// launches 6k..6k+5 for every k >= 1.  The vectors are the plan's own (b^ in T1, x^ in T2).
smr_status ensure_steady_graph(const Plan &p, double *Xh, const double *Bh) {
  if (p.steady6) return SMR_OK;
  hipStream_t cs = plan_capture_stream(p);
  if (!cs) return fail(SMR_EDEVICE, "no capture stream");
  Ctx cc{&p, cs};
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int j = 6; j < 12 && e == hipSuccess; ++j) {
    if (!p.const_coef) e = launch_kslice(cc, 1, j, Xh, Bh);
    if (e == hipSuccess) e = launch_spec(cc, 2, j, Xh, Bh);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return fail(SMR_EDEVICE, "capturing the steady iterations failed: %s",
                hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(SMR_EDEVICE, "instantiating the steady iterations failed: %s", hipGetErrorString(e3));
  p.steady6 = ex;
  return SMR_OK;
}

// Host-side state of the batched solves on one device: the capture stream, the captured steady
// iterations (keyed by the batch workspace address and the class layout of the launches; a few
// recent layouts are kept) and the pinned status snapshots.  Every batched call holds `mu` from
// start to end, so concurrent batched calls on one device run one after another and never
// share a snapshot buffer, a capture or a cached graph while another call uses it.
struct BatchState {
  std::mutex mu;
  hipStream_t cs = nullptr;
  struct Entry {
    std::vector<long> key;
    hipGraphExec_t ex;
  };
  std::vector<Entry> cache;
  Scal *snap = nullptr;        // two slots of `cap` instances
  int cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // side streams and events of the captured iterations, whose size classes of one phase run
  // on parallel branches (made on first use)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> cev;
};
BatchState &batch_state() {
  static std::mutex mu;
  static std::map<int, BatchState> per_device;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  return per_device[dev];   // std::map never moves its elements
}

// The steady-iteration graph of a batch layout (captured on first use); bs.mu must be held.
template <typename F>
hipGraphExec_t batch_graph(BatchState &bs, const std::vector<long> &key, F &&enqueue) {
  for (const BatchState::Entry &en : bs.cache)
    if (en.key == key) return en.ex;
  if (!bs.cs && hipStreamCreateWithFlags(&bs.cs, hipStreamNonBlocking) != hipSuccess) bs.cs = nullptr;
  if (!bs.cs || hipStreamBeginCapture(bs.cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  const hipError_t e = enqueue(bs.cs);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(bs.cs, &g);
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess && e2 == hipSuccess && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
  if (g) hipGraphDestroy(g);
  if (!ex) return nullptr;
  if (bs.cache.size() >= 8) {
    hipGraphExecDestroy(bs.cache.front().ex);   // no other call can be replaying it (bs.mu)
    bs.cache.erase(bs.cache.begin());
  }
  bs.cache.push_back(BatchState::Entry{key, ex});
  return ex;
}

// Pinned host status snapshots for `count` instances (two slots); bs.mu must be held, and the
// previous call's copies into the old buffer have completed (each call synchronises before
// it returns).
bool batch_snapshots(BatchState &bs, int count) {
  if (count > bs.cap) {
    if (bs.snap) hipHostFree(bs.snap);
    bs.snap = nullptr;
    bs.cap = 0;
    if (hipHostMalloc((void **)&bs.snap, 2 * sizeof(Scal) * (size_t)count, hipHostMallocDefault) == hipSuccess)
      bs.cap = count;
  }
  for (hipEvent_t &e : bs.ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
  return bs.snap && bs.ev[0] && bs.ev[1];
}

// Constant coefficients: the whole MINRES runs in the spatial sine basis with one fused
// kernel per iteration; b and x0 are transformed on entry, the iterate on exit.
// x0 == NULL: zero initial guess (the initialising launch writes x = 0 in the sine basis)
smr_status minres_spectral(const Plan &p, hipStream_t s, const double *b, const double *x0, double *x, double rtol,
                           int maxit, smr_info *info) {
  Ctx c{&p, s};
  double *Bh = p.T1, *Xh = p.T2;
  smr_status st = to_sine_basis(p, s, b, Bh);
  if (st != SMR_OK) return st;
  if (x0) {
    st = to_sine_basis(p, s, x0, Xh);
    if (st != SMR_OK) return st;
  }
  Scal h{};
  const bool ext = !p.const_coef;   // variable a: (T z)^ from the per-level matvec
  if (ext && x0) LAUNCH(PROF_KSLICE, launch_kslice(c, 0, 0, Xh, Bh));
  LAUNCH(PROF_SPEC, launch_spec(c, 0, 0, Xh, Bh, x0 == nullptr, rtol, maxit));
  const Profiler::Mark m0 = g_prof.mark();
  st = ensure_snapshots(p);
  if (st != SMR_OK) return st;
  // launches j >= 6 replay six captured iterations, except while profiling a variable-
  // coefficient solve (a replay's events could not separate its two kernels)
  const bool graph = !(g_prof.on && ext) && ensure_steady_graph(p, Xh, Bh) == SMR_OK;
  int issued = 0;                   // launches j = 1..issued enqueued
  const int last = maxit + 2;       // launch maxit + 2 takes the stop decision on iteration maxit
  int pend[2], npend = 0, slot_next = 0;
  long pend_seq[2], seq = 0;        // order of the enqueued snapshots
  // Stop prediction.  Every snapshot carries |eta| / gamma_1, the relative residual in the
  // P^{-1} norm (monotone in MINRES), and, once true residuals are evaluated, their ratio to
  // it.  From its decay between the last two snapshots and the latest ratio the host predicts
  // the stopping iteration, enqueues only the launches up to it (two spare) and then waits for
  // the snapshot after them before enqueueing more.  A wrong prediction costs a host round
  // trip, never a result: the device takes the stop decision itself.
  // The transform of the result back from the sine basis follows those launches, gated on the
  // stopped state, so that a right prediction costs no round trip at the end either; it ran iff
  // the snapshot after it (and every later one) read a stopped state.
  int e_it[2] = {-1, -1}, seen_nres = 1;
  double e_v[2] = {0.0, 0.0}, ratio = 1.0;
  int spent = 1 << 30;              // last launch of the prediction, once enqueued
  long spent_seq = -1;              // the snapshot taken right after it
  bool short_pred = false;          // that snapshot or a later one read RUNNING
  const bool ahead_ok = kslice_supported(&p) && Xh != x;   // the one-pass transform
  bool ahead = false;
  Ctx cx{&p, s};
  // enqueue up to `cap` launches (a captured chunk of six when aligned) and a snapshot of the
  // state after them (pinned host copy + event)
  auto enqueue_next = [&](int cap) -> smr_status {
    const bool aligned = issued >= 5 && (issued + 1) % 6 == 0;
    if (graph && aligned && cap >= 6 && last - issued >= 6) {
      ProfScope ps(PROF_SPEC, s, 6);
      HIP_TRY(hipGraphLaunch(p.steady6, s));
      issued += 6;
    } else {
      const int todo = std::min(std::min(cap, issued < 5 ? 5 - issued : 6), last - issued);
      for (int it = 0; it < todo; ++it) {
        const int j = issued + it + 1;
        if (ext) LAUNCH(PROF_KSLICE, launch_kslice(c, 1, j, Xh, Bh));
        LAUNCH(PROF_SPEC, launch_spec(c, j == 1 ? 1 : 2, j, Xh, Bh));
      }
      issued += todo;
    }
    if (spent_seq < 0 && issued >= spent) {
      if (ahead_ok) {
        LAUNCH(PROF_DST, launch_dst2d(cx, Xh, x, p.ld, p.m, p.sc + (issued & 1)));
        ahead = true;
      }
      spent_seq = seq;
    }
    HIP_TRY(hipMemcpyAsync(&p.snap[slot_next], p.sc + (issued & 1), sizeof(Scal), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(p.snap_ev[slot_next], s));
    pend_seq[npend] = seq++;
    pend[npend++] = slot_next;
    slot_next ^= 1;
    return SMR_OK;
  };
  auto predicted_cap = [&]() -> int {
    if (short_pred) return 6;                            // the prediction fell short: whole chunks
    if (spent_seq >= 0) return 0;                        // wait for its outcome
    if (e_it[0] < 0 || e_it[1] <= e_it[0] || !(e_v[1] > 0.0) || !(e_v[0] > e_v[1])) return 6;
    const double rho = std::pow(e_v[1] / e_v[0], 1.0 / (e_it[1] - e_it[0]));
    if (!(rho > 0.0 && rho < 1.0)) return 6;
    const double est = ratio * e_v[1];                   // true relative residual, estimated
    const double more = est <= rtol ? 0.0 : std::ceil(std::log(rtol / est) / std::log(rho));
    if (!(more < 1e6)) return 6;
    const int reach = e_it[1] + (int)more + 2 + 2;      // launch stop + 2 decides; two spare
    if (reach - issued > 6) return 6;
    // the last chunk: a captured one whole where one is due (launches enqueued one by one
    // behind a graph replay start late), else the launches up to the predicted stop
    const bool aligned = graph && issued >= 5 && (issued + 1) % 6 == 0 && last - issued >= 6;
    spent = aligned ? issued + 6 : std::max(reach, issued + 1);
    return spent - issued;
  };
  // keep one chunk in flight ahead of the status being checked, so the device never waits
  st = enqueue_next(6);
  if (st != SMR_OK) return st;
  for (;;) {
    if (issued < last && npend < 2) {
      int cap = predicted_cap();
      if (npend == 0) cap = std::max(cap, 1);          // the solve is still running
      if (cap > 0) {
        st = enqueue_next(cap);
        if (st != SMR_OK) return st;
      }
    }
    const int slot = pend[0];
    const long sq = pend_seq[0];
    pend[0] = pend[1];
    pend_seq[0] = pend_seq[1];
    --npend;
    HIP_TRY(hipEventSynchronize(p.snap_ev[slot]));
    h = p.snap[slot];
    if (h.status == RUNNING && spent_seq >= 0 && sq >= spent_seq) short_pred = true;
    if (h.status != RUNNING) break;
    if (npend == 0 && issued >= last) break;
    const double pr = h.gamma1 > 0.0 ? std::fabs(h.eta) / h.gamma1 : 0.0;
    if (h.iter > e_it[1]) {
      e_it[0] = e_it[1];
      e_v[0] = e_v[1];
      e_it[1] = h.iter;
      e_v[1] = pr;
    }
    if (h.nres > seen_nres && pr > 0.0) {               // a true residual of the steady phase
      ratio = h.relres / pr;
      seen_nres = h.nres;
    }
  }
  // h is final: a stopped state is passed on unchanged by the launches after the decision, and
  // the iteration-limit exit read the snapshot taken after the last launch
  if (g_prof.on) {   // keep the records of the launches that did work (j = 1 .. iter + 1)
    g_prof.keep_launches(m0, PROF_SPEC, std::min(issued, h.iter + 1));
    if (ext) g_prof.keep_launches(m0, PROF_KSLICE, std::min(issued, h.iter + 1));
  }
  const bool ahead_ran = ahead && !short_pred && h.status != RUNNING;
  if (h.status == DONE_CONV && h.bnorm == 0.0) {
    LAUNCH(PROF_VEC, launch_zero(c, x, p.len));
  } else if (!ahead_ran) {
    st = from_sine_basis(p, s, Xh, x);
    if (st != SMR_OK) return st;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return finish_info(h, maxit, info, p.spec_c);
}

const double *scal_field(const Plan &p, size_t off) { return (const double *)((const char *)p.sc + off); }

// MINRES on (Y T) x = Y b from the initial x; b unpermuted.
smr_status minres(const Plan &p, hipStream_t s, const double *b, const double *x0, double *x, double rtol, int maxit,
                  smr_info *info) {
  Ctx c{&p, s};
  if (!x0) LAUNCH(PROF_VEC, launch_zero(c, x, p.len));
  else if (x0 != x) HIP_TRY(hipMemcpyAsync(x, x0, p.len * sizeof(double), hipMemcpyDeviceToDevice, s));
  Scal h{};
  h.rtol = rtol;
  h.maxit = maxit;
  h.status = RUNNING;
  HIP_TRY(hipMemcpyAsync(p.sc, &h, sizeof(Scal), hipMemcpyHostToDevice, s));
  LAUNCH(PROF_VEC, launch_zero(c, p.V[0], p.vlen));
  LAUNCH(PROF_VEC, launch_zero(c, p.W[0], p.vlen));
  LAUNCH(PROF_VEC, launch_zero(c, p.W[1], p.vlen));
  double *part = p.part, *part2 = p.part + 2 * kRedSlots;
  int nb = 0, nb2 = 0;
  // v_1 = Y b - Y T x0, ||v_1||^2, ||b||^2
  LAUNCH(PROF_STENCIL, launch_apply_YT(c, x, nullptr, p.V[1], b, part, &nb, nullptr));
  const bool f32 = p.pprec == SMR_FP32;
  smr_status st = apply_pinv(p, s, p.V[1], p.Z[0], part2, &nb2, nullptr, f32, plan_bufs(p));
  if (st != SMR_OK) return st;
  LAUNCH(PROF_SCALAR, launch_scalar_step(c, 0, part, nb, part2, nb2));
  int cv = 1, cz = 0, cw = 1;   // v_j = V[cv], v_{j-1} = V[1-cv]; z_j = Z[cz]; w_{j-1} = W[cw], w_{j-2} = W[1-cw]
  const Scal *gate = p.sc;
  const double *zs = scal_field(p, offsetof(Scal, zs));
  int issued = 0;
  int chunk = 4;
  std::vector<Profiler::Mark> marks;
  for (;;) {
    HIP_TRY(hipMemcpyAsync(&h, p.sc, sizeof(Scal), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h.status != RUNNING || issued >= maxit) break;
    const int todo = std::min(chunk, maxit - issued);
    for (int it = 0; it < todo; ++it) {
      marks.push_back(g_prof.mark());
      double *vj = p.V[cv], *vo = p.V[1 - cv], *zj = p.Z[cz], *zn = p.Z[1 - cz];
      double *w1 = p.W[cw], *w2 = p.W[1 - cw];
      LAUNCH(PROF_STENCIL, launch_apply_YT(c, zj, zs, p.Q, nullptr, part, &nb, gate));
      LAUNCH(PROF_SCALAR, launch_scalar_step(c, 1, part, nb, nullptr, 0));
      LAUNCH(PROF_VEC, launch_vupdate(c, p.Q, vj, vo, gate));
      st = apply_pinv(p, s, vo, zn, part2, &nb2, gate, f32, plan_bufs(p));
      if (st != SMR_OK) return st;
      LAUNCH(PROF_SCALAR, launch_scalar_step(c, 2, part2, nb2, part2, nb2));
      LAUNCH(PROF_VEC, launch_wxupdate(c, zj, w2, w1, x, gate));
      LAUNCH(PROF_STENCIL, launch_apply_YT(c, x, nullptr, nullptr, b, part, &nb, gate));
      LAUNCH(PROF_SCALAR, launch_scalar_step(c, 3, part, nb, nullptr, 0));
      cv ^= 1;
      cz ^= 1;
      cw ^= 1;
    }
    issued += todo;
    chunk = std::min(chunk * 2, 16);
  }
  if (g_prof.on && h.iter < (int)marks.size()) g_prof.truncate(marks[h.iter]);
  if (h.status == DONE_CONV && h.bnorm == 0.0) LAUNCH(PROF_VEC, launch_zero(c, x, p.len));
  HIP_TRY(hipStreamSynchronize(s));
  smr_status res = SMR_OK;
  switch (h.status) {
    case DONE_CONV: res = SMR_OK; break;
    case DONE_NOTSPD: res = fail(SMR_ENOTSPD, "preconditioner not SPD on the residual (gamma^2 <= 0 or not finite)"); break;
    case DONE_BREAKDOWN: res = fail(SMR_EBREAKDOWN, "MINRES breakdown (alpha1 = 0)"); break;
    default: res = fail(SMR_ENOTCONV, "maxit = %d reached, relres = %g", maxit, h.relres); break;
  }
  if (info) {
    info->iters = h.iter;
    info->status = res;
    info->relres_true = h.bnorm == 0.0 ? 0.0 : h.relres;
    info->relres_prec = h.gamma1 > 0.0 ? std::fabs(h.eta) / h.gamma1 : 0.0;
    info->res_evals = h.iter + 1;      // the physical-basis iteration evaluates every one
    info->tile_cols = 0;
  }
  return res;
}

}  // namespace
}  // namespace smr

extern "C" {

smr_status smr_pinv_variant(const smr_plan *plan, int32_t *variant) {
  if (!plan || !variant) return fail(SMR_EINVAL, "plan and variant must be non-NULL");
  *variant = plan->p.pinv_var;
  return SMR_OK;
}

smr_status smr_matvec_tiles(const smr_plan *plan, int32_t *tiled) {
  if (!plan || !tiled) return fail(SMR_EINVAL, "plan and tiled must be non-NULL");
  *tiled = plan->p.ks_split ? 1 : 0;
  return SMR_OK;
}

smr_status smr_tune_stats(int64_t *entries, int64_t *hits, int64_t *misses) {
  if (!entries || !hits || !misses) return fail(SMR_EINVAL, "NULL argument");
  long e = 0, h = 0, m = 0;
  tune_stats(&e, &h, &m);
  *entries = e;
  *hits = h;
  *misses = m;
  return SMR_OK;
}

smr_status smr_tune_reset(void) {
  tune_clear();
  return SMR_OK;
}

smr_status smr_tile_cols(const smr_plan *plan, int32_t *cols) {
  if (check_plan(plan) != SMR_OK) return SMR_EINVAL;
  if (!cols) return fail(SMR_EINVAL, "cols is NULL");
  *cols = use_spectral(plan->p) ? spec_cols(&plan->p) : 0;
  return SMR_OK;
}


smr_status smr_build_rhs(const smr_plan *pl, const double *f, const double *u0, double *b, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (pl->p.scheme != SMR_THETA) return fail(SMR_EINVAL, "smr_build_rhs is defined for the theta scheme");
  if (!f || !b) return fail(SMR_EINVAL, "f and b must be non-NULL");
  Ctx c{&pl->p, (hipStream_t)stream};
  LAUNCH(PROF_STENCIL, launch_build_rhs(c, f, u0, b));
  return SMR_OK;
}

smr_status smr_apply_A(const smr_plan *pl, const double *x, double *y, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (!x || !y || x == y) return fail(SMR_EINVAL, "x and y must be distinct non-NULL device pointers");
  Ctx c{&pl->p, (hipStream_t)stream};
  LAUNCH(PROF_STENCIL, launch_apply_YT(c, x, nullptr, y, nullptr, nullptr, nullptr, nullptr));
  return SMR_OK;
}

smr_status smr_apply_P_inv(const smr_plan *pl, const double *v, double *z, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (!v || !z) return fail(SMR_EINVAL, "v and z must be non-NULL");
  return apply_pinv(pl->p, (hipStream_t)stream, v, z, nullptr, nullptr, nullptr, false, plan_bufs(pl->p));
}

}  // extern "C"

// ---------------------------------------------------------------- static scratch
// Intermediate vectors of smr_apply_P_inv_static: a library-owned array in device memory, one
// copy per GPU, alive until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name only stands in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[SMR_STATIC_SCRATCH_BYTES];

namespace smr {
namespace {

smr_status static_scratch(double **out) {
  static std::mutex mu;
  static std::map<int, void *> ptr;   // device -> address of its copy of `scratch`
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptr.find(dev);
  if (it == ptr.end()) {
    void *a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !a)
      return fail(SMR_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    it = ptr.emplace(dev, a).first;
  }
  *out = (double *)it->second;
  return SMR_OK;
}

}  // namespace
}  // namespace smr

extern "C" {

smr_status smr_apply_P_inv_static(const smr_plan *pl, const double *v, double *z, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (!v || !z) return fail(SMR_EINVAL, "v and z must be non-NULL");
  const Plan &p = pl->p;
  const int nvec = p.precond == SMR_P_H ? 2 : p.precond == SMR_P_THETA_CHEB ? 4 : 0;
  const size_t vbytes = align256(p.len * sizeof(double));
  if ((size_t)nvec * vbytes > (size_t)SMR_STATIC_SCRATCH_BYTES)
    return fail(SMR_EINVAL, "P^{-1} of this plan needs %d vectors of %zu bytes, more than the %llu bytes of static "
                "scratch", nvec, vbytes, (unsigned long long)SMR_STATIC_SCRATCH_BYTES);
  double *base = nullptr;
  st = static_scratch(&base);
  if (st != SMR_OK) return st;
  const size_t stride = vbytes / sizeof(double);
  const PinvBufs tb{base, base + stride, nvec == 4 ? base + 2 * stride : nullptr, nvec == 4 ? base + 3 * stride : nullptr};
  return apply_pinv(p, (hipStream_t)stream, v, z, nullptr, nullptr, nullptr, false, tb);
}

smr_status smr_minres_solve(const smr_plan *pl, const double *b, const double *x0, double *x, double rtol,
                            int32_t maxit, smr_info *info, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (!b || !x) return fail(SMR_EINVAL, "b and x must be non-NULL");
  if (b == x) return fail(SMR_EINVAL, "b and x must be distinct");
  if (!(rtol > 0.0) || maxit < 0) return fail(SMR_EINVAL, "need rtol > 0 and maxit >= 0");
  if (use_spectral(pl->p)) return minres_spectral(pl->p, (hipStream_t)stream, b, x0, x, rtol, maxit, info);
  return minres(pl->p, (hipStream_t)stream, b, x0, x, rtol, maxit, info);
}

smr_status smr_batch_workspace_size(int32_t count, const smr_plan *const *plans, size_t *bytes) {
  if (count < 0 || (count > 0 && !plans) || !bytes) return fail(SMR_EINVAL, "bad batch arguments");
  const size_t c1 = (size_t)std::max(count, 1);
  *bytes = align256(sizeof(SpecP) * c1) + align256(sizeof(Scal) * c1) + align256(sizeof(KsP) * c1);
  return SMR_OK;
}

}  // extern "C"

namespace smr {
namespace {

// Every instance of a batch iterates in its own plan's vectors and scalars, so a plan may
// appear only once.
smr_status check_distinct_plans(int count, const smr_plan *const *plans) {
  std::unordered_set<const smr_plan *> seen;
  for (int i = 0; i < count; ++i)
    if (!seen.insert(plans[i]).second) return fail(SMR_EINVAL, "instance %d: plan repeated within the batch", i);
  return SMR_OK;
}

// Times steady fused launches of a group of batch instances at each column-tile width (on
// their own workspaces, from a running state that never converges, through the batch's
// descriptor table) and returns the fastest: 32 unless 16 (or 64, for hp <= 64, or 128 in float32) is at least
// 5% faster.
smr_status batch_width_tune(hipStream_t s, const smr_plan *const *plans, const std::vector<int> &ids, int hp,
                            int pprec, int taps, SpecP *d_table, int *width) {
  const int cand[3] = {32, 16, 64};
  const int ncand = spec_cols_ok(hp, 64, pprec) ? 3 : 2;
  float best[3] = {1e30f, 1e30f, 1e30f};
  std::vector<SpecP> t(ids.size());
  // three interleaved rounds, the fastest of each width kept (steadier than one round)
  for (int rep = 0; rep < 3; ++rep) {
    for (int k = 0; k < ncand; ++k) {
      int blocks = 0;
      for (size_t q = 0; q < ids.size(); ++q) {
        const Plan &p = plans[ids[q]]->p;
        t[q] = spec_desc(&p, p.T2, p.T1, cand[k]);
        t[q].rtiles = 0;
        t[q].tile0 = blocks;
        blocks += t[q].tiles;
        HIP_TRY(spec_tune_state(&p, s, t[q]));
      }
      HIP_TRY(hipMemcpyAsync(d_table, t.data(), sizeof(SpecP) * t.size(), hipMemcpyHostToDevice, s));
      // a steady launch with j = 7 reads slot 0 and writes slot 1: repeated launches start alike
      float ms = 0.0f;
      HIP_TRY(tune_time(s, 4, [&]() {
        return launch_spec_multi(s, d_table, (int)ids.size(), blocks, hp, cand[k], pprec, taps, 2, 7);
      }, &ms));
      best[k] = std::min(best[k], ms);
    }
  }
  int arg = 0;
  for (int k = 1; k < ncand; ++k)
    if (best[k] < 0.95f * best[0] && best[k] < best[arg]) arg = k;
  *width = cand[arg];
  return SMR_OK;
}

smr_status solve_batched_locked(BatchState &bst, int32_t count, const smr_plan *const *plans, const double *const *b,
                                const double *const *x0, double *const *x, double rtol, int32_t maxit, void *d_ws,
                                smr_info *infos, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  SpecP *d_table = (SpecP *)d_ws;
  const size_t c1 = (size_t)std::max(count, 1);
  Scal *d_scal = (Scal *)((char *)d_ws + align256(sizeof(SpecP) * c1));
  KsP *d_ks = (KsP *)((char *)d_ws + align256(sizeof(SpecP) * c1) + align256(sizeof(Scal) * c1));
  // sine-basis instances, grouped by (time-size class, transform precision)
  std::vector<int> spec_ids, general_ids;
  for (int i = 0; i < count; ++i) (use_spectral(plans[i]->p) ? spec_ids : general_ids).push_back(i);
  // kernel instantiation of an instance's fused launch: 3 time taps (theta, BDF2) or 5
  auto taps_of = [](const Plan &p) { return p.taps <= 3 ? 3 : 5; };
  // Column-tile width per instance: a width forced on the plan stays; the other instances of
  // a (time-size class, precision, time taps) group share one width, timed on the group's own
  // workspaces the first time the group's shape is seen on the device (then cached), before
  // any of this call's data enters them.
  std::vector<int> cols(count, 0);
  {
    auto forced = [](const Plan &p) { return (p.flags & (SMR_FLAG_TILE16 | SMR_FLAG_TILE32 | SMR_FLAG_TILE64)) != 0; };
    struct Group {
      int hp, pprec, taps;
      std::vector<int> ids;
    };
    std::vector<Group> groups;
    for (int i : spec_ids) {
      const Plan &p = plans[i]->p;
      if (forced(p)) { cols[i] = p.spec_c; continue; }
      if (!spec_cols_ok(p.hp, 32)) { cols[i] = 16; continue; }
      Group *g = nullptr;
      for (Group &h : groups)
        if (h.hp == p.hp && h.pprec == p.pprec && h.taps == taps_of(p)) g = &h;
      if (!g) {
        groups.push_back(Group{p.hp, p.pprec, taps_of(p), {}});
        g = &groups.back();
      }
      g->ids.push_back(i);
    }
    for (const Group &g : groups) {
      long tiles16 = 0, nvar = 0;
      for (int i : g.ids) {
        tiles16 += (plans[i]->p.m + 15) / 16;
        nvar += plans[i]->p.const_coef ? 0 : 1;
      }
      const std::vector<long> key{TUNE_BATCH_WIDTH, g.hp, g.pprec, g.taps, (long)g.ids.size(), tiles16, nvar};
      int w = 0;
      if (!tune_get(key, &w)) {
        const smr_status st = batch_width_tune(s, plans, g.ids, g.hp, g.pprec, g.taps, d_table, &w);
        if (st != SMR_OK) return st;
        tune_put(key, w);
      }
      for (int i : g.ids) cols[i] = w;
    }
  }
  std::stable_sort(spec_ids.begin(), spec_ids.end(), [&](int a, int c) {
    const Plan &pa = plans[a]->p, &pc = plans[c]->p;
    if (pa.hp != pc.hp) return pa.hp < pc.hp;
    if (taps_of(pa) != taps_of(pc)) return taps_of(pa) < taps_of(pc);
    return cols[a] != cols[c] ? cols[a] < cols[c] : pa.pprec < pc.pprec;
  });
  struct Class { int first, count, blocks, hp, cols, pprec, taps; };
  std::vector<Class> classes;
  std::vector<SpecP> table(spec_ids.size());
  for (size_t k = 0; k < spec_ids.size(); ++k) {
    const Plan &p = plans[spec_ids[k]]->p;
    const int c = cols[spec_ids[k]];
    if (classes.empty() || classes.back().hp != p.hp || classes.back().cols != c || classes.back().pprec != p.pprec ||
        classes.back().taps != taps_of(p))
      classes.push_back(Class{(int)k, 0, 0, p.hp, c, p.pprec, taps_of(p)});
    Class &cl = classes.back();
    table[k] = spec_desc(&p, p.T2, p.T1, c);
    table[k].rtiles = 0;   // batched launches read every tile's partials (no grouped reduction)
    table[k].tile0 = cl.blocks;
    cl.blocks += table[k].tiles;
    cl.count += 1;
  }
  const int ns = (int)spec_ids.size();
  // variable-coefficient sine-basis instances: per-level matvec, grouped by (N + 1, precision)
  std::vector<int> var_ids;
  for (int i : spec_ids)
    if (!plans[i]->p.const_coef) var_ids.push_back(i);
  std::stable_sort(var_ids.begin(), var_ids.end(), [&](int a, int c) {
    const Plan &pa = plans[a]->p, &pc = plans[c]->p;
    return pa.L != pc.L ? pa.L < pc.L : pa.pprec != pc.pprec ? pa.pprec < pc.pprec : pa.ks_split < pc.ks_split;
  });
  struct KClass { int first, count, blocks, L, pprec; bool split; };
  std::vector<KClass> kclasses;
  std::vector<KsP> ktable(var_ids.size());
  for (size_t k = 0; k < var_ids.size(); ++k) {
    const Plan &p = plans[var_ids[k]]->p;
    if (kclasses.empty() || kclasses.back().L != p.L || kclasses.back().pprec != p.pprec ||
        kclasses.back().split != p.ks_split)
      kclasses.push_back(KClass{(int)k, 0, 0, p.L, p.pprec, p.ks_split});
    KClass &cl = kclasses.back();
    ktable[k] = kslice_desc(&p, p.T2, p.T1);
    ktable[k].blk0 = cl.blocks;
    cl.blocks += p.n;
    cl.count += 1;
  }
  smr_status first_bad = SMR_OK;
  bool any_guess_ext = false;
  if (ns > 0) {
    for (int k = 0; k < ns; ++k) {
      const Plan &p = plans[spec_ids[k]]->p;
      smr_status st = to_sine_basis(p, s, b[spec_ids[k]], p.T1);
      if (st != SMR_OK) return st;
      const double *g0 = x0 ? x0[spec_ids[k]] : nullptr;
      if (g0) {
        st = to_sine_basis(p, s, g0, p.T2);
        if (st != SMR_OK) return st;
        any_guess_ext |= !p.const_coef;
      }
      table[k].x0zero = g0 == nullptr;
      table[k].rtol = rtol;
      table[k].maxit = maxit;
    }
    HIP_TRY(hipMemcpyAsync(d_table, table.data(), sizeof(SpecP) * ns, hipMemcpyHostToDevice, s));
    if (!ktable.empty())
      HIP_TRY(hipMemcpyAsync(d_ks, ktable.data(), sizeof(KsP) * ktable.size(), hipMemcpyHostToDevice, s));
    Ctx c0{&plans[spec_ids[0]]->p, s};
    Ctx &c = c0;
    // (T x0)^ is needed only for a given guess (zero-guess instances ignore it)
    if (any_guess_ext)
      for (const KClass &cl : kclasses)
        LAUNCH(PROF_KSLICE, launch_kslice_multi(s, d_ks + cl.first, cl.count, cl.blocks, cl.L, cl.pprec, 0, 0, cl.split));
    for (const Class &cl : classes)
      LAUNCH(PROF_SPEC, launch_spec_multi(s, d_table + cl.first, cl.count, cl.blocks, cl.hp, cl.cols, cl.pprec, cl.taps, 0, 0));
    // one iteration j: the per-level matvec of every N class, then the fused launch of every
    // time-size class
    // One captured iteration j: the per-level matvec of every N class, then the fused launch of
    // every time-size class.  The classes of one phase touch disjoint instances, so each runs
    // on a branch of its own (side streams forked from and joined back into the capture
    // stream), letting a small class fill the compute units a large one leaves idle; the
    // fused phase waits for every matvec class, the next iteration for every fused class.
    // the side streams and events are made before the capture begins (one event per fork and
    // per join of every phase of the six iterations)
    {
      const size_t nside = std::max(kclasses.size(), classes.size());
      while (bst.side.size() + 1 < nside) {
        hipStream_t st = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        bst.side.push_back(st);
      }
      while (bst.cev.size() < 6 * (kclasses.size() + classes.size())) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        bst.cev.push_back(e);
      }
    }
    size_t nev = 0;
    auto next_event = [&](hipEvent_t *out) -> hipError_t {
      if (nev >= bst.cev.size()) return hipErrorInvalidValue;
      *out = bst.cev[nev++];
      return hipSuccess;
    };
    auto phase = [&](hipStream_t cs, int nbranch, auto launch_one) -> hipError_t {
      hipError_t e = hipSuccess;
      if (nbranch <= 1) return nbranch == 1 ? launch_one(cs, 0) : hipSuccess;
      hipEvent_t fork = nullptr;
      if (e == hipSuccess) e = next_event(&fork);
      if (e == hipSuccess) e = hipEventRecord(fork, cs);
      for (int c = 1; c < nbranch && e == hipSuccess; ++c) e = hipStreamWaitEvent(bst.side[c - 1], fork, 0);
      for (int c = 0; c < nbranch && e == hipSuccess; ++c) e = launch_one(c == 0 ? cs : bst.side[c - 1], c);
      for (int c = 1; c < nbranch && e == hipSuccess; ++c) {
        hipEvent_t join = nullptr;
        e = next_event(&join);
        if (e == hipSuccess) e = hipEventRecord(join, bst.side[c - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, join, 0);
      }
      return e;
    };
    auto iteration_par = [&](hipStream_t cs, int j) -> hipError_t {
      hipError_t e = phase(cs, (int)kclasses.size(), [&](hipStream_t st, int c) {
        const KClass &cl = kclasses[c];
        return launch_kslice_multi(st, d_ks + cl.first, cl.count, cl.blocks, cl.L, cl.pprec, 1, j, cl.split);
      });
      if (e == hipSuccess)
        e = phase(cs, (int)classes.size(), [&](hipStream_t st, int c) {
          const Class &cl = classes[c];
          return launch_spec_multi(st, d_table + cl.first, cl.count, cl.blocks, cl.hp, cl.cols, cl.pprec, cl.taps,
                                   j == 1 ? 1 : 2, j);
        });
      return e;
    };
    // steady iterations j >= 6 replay a captured graph of six (cached by workspace and class
    // layout; the tables it reads are re-uploaded above on every call), except while profiling
    hipGraphExec_t g6 = nullptr;
    if (!g_prof.on) {
      // the descriptor tables' places in the workspace depend on the instance count as well
      std::vector<long> key{(long)(uintptr_t)d_ws, (long)count};
      for (const KClass &cl : kclasses)
        key.insert(key.end(), {0, cl.first, cl.count, cl.blocks, cl.L, cl.pprec, cl.split ? 1L : 0L});
      for (const Class &cl : classes)
        key.insert(key.end(), {1, cl.first, cl.count, cl.blocks, cl.hp, cl.cols, cl.pprec, cl.taps});
      g6 = batch_graph(bst, key, [&](hipStream_t cs) {
        hipError_t e = hipSuccess;
        for (int j = 6; j < 12 && e == hipSuccess; ++j) e = iteration_par(cs, j);
        return e;
      });
    }
    if (!batch_snapshots(bst, ns)) return fail(SMR_EDEVICE, "pinned status buffer");
    struct {
      Scal *h;
      int cap;
      hipEvent_t *ev;
    } bs{bst.snap, bst.cap, bst.ev};
    std::vector<Scal> hs(ns);
    int issued = 0;
    const int last = maxit + 2;
    int pend[2], npend = 0, slot_next = 0;
    auto enqueue_next = [&]() -> smr_status {
      if (issued < 5 || !g6) {
        const int todo = std::min(issued < 5 ? 5 - issued : 6, last - issued);
        for (int it = 0; it < todo; ++it) {
          const int j = issued + it + 1;
          for (const KClass &cl : kclasses)
            LAUNCH(PROF_KSLICE, launch_kslice_multi(s, d_ks + cl.first, cl.count, cl.blocks, cl.L, cl.pprec, 1, j, cl.split));
          for (const Class &cl : classes)
            LAUNCH(PROF_SPEC, launch_spec_multi(s, d_table + cl.first, cl.count, cl.blocks, cl.hp, cl.cols, cl.pprec, cl.taps,
                                                j == 1 ? 1 : 2, j));
        }
        issued += todo;
      } else {
        HIP_TRY(hipGraphLaunch(g6, s));
        issued += 6;
      }
      HIP_TRY(launch_gather_scal(s, d_table, ns, issued & 1, d_scal));
      HIP_TRY(hipMemcpyAsync(bs.h + (size_t)slot_next * bs.cap, d_scal, sizeof(Scal) * ns, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(bs.ev[slot_next], s));
      pend[npend++] = slot_next;
      slot_next ^= 1;
      return SMR_OK;
    };
    smr_status st0 = enqueue_next();
    if (st0 != SMR_OK) return st0;
    int slot = 0;
    for (;;) {
      if (issued < last && npend < 2) {
        st0 = enqueue_next();
        if (st0 != SMR_OK) return st0;
      }
      slot = pend[0];
      pend[0] = pend[1];
      --npend;
      HIP_TRY(hipEventSynchronize(bs.ev[slot]));
      bool running = false;
      for (int k = 0; k < ns; ++k) running |= (bs.h[(size_t)slot * bs.cap + k].status == RUNNING);
      if (!running) break;
      if (npend == 0 && issued >= last) break;
    }
    // the snapshot just read is final: a stopped instance's state is passed on unchanged, and
    // the iteration-limit exit read the snapshot taken after the last launch
    std::copy(bs.h + (size_t)slot * bs.cap, bs.h + (size_t)slot * bs.cap + ns, hs.begin());
    for (int k = 0; k < ns; ++k) {
      const int i = spec_ids[k];
      const Plan &p = plans[i]->p;
      Ctx ci{&p, s};
      Ctx &c = ci;
      if (hs[k].status == DONE_CONV && hs[k].bnorm == 0.0) {
        LAUNCH(PROF_VEC, launch_zero(c, x[i], p.len));
      } else {
        smr_status st = from_sine_basis(p, s, p.T2, x[i]);
        if (st != SMR_OK) return st;
      }
      smr_status st = finish_info(hs[k], maxit, &infos[i], cols[i]);
      if (st != SMR_OK && first_bad == SMR_OK) first_bad = st;
    }
    HIP_TRY(hipStreamSynchronize(s));
  }
  for (int i : general_ids) {
    smr_status st = minres(plans[i]->p, s, b[i], x0 ? x0[i] : nullptr, x[i], rtol, maxit, &infos[i]);
    if (st != SMR_OK && first_bad == SMR_OK) first_bad = st;
  }
  return first_bad;
}

}  // namespace
}  // namespace smr

extern "C" {

smr_status smr_minres_solve_batched(int32_t count, const smr_plan *const *plans, const double *const *b,
                                    const double *const *x0, double *const *x, double rtol, int32_t maxit,
                                    void *d_ws, size_t ws_bytes, smr_info *infos, void *stream) {
  if (count < 0 || (count > 0 && (!plans || !b || !x || !infos))) return fail(SMR_EINVAL, "bad batch arguments");
  if (!(rtol > 0.0) || maxit < 0) return fail(SMR_EINVAL, "need rtol > 0 and maxit >= 0");
  size_t need = 0;
  smr_batch_workspace_size(count, plans, &need);
  if (count > 0 && (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < need))
    return fail(SMR_EWORKSPACE, "batch workspace missing, misaligned or smaller than %zu bytes", need);
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !b[i] || !x[i]) return fail(SMR_EINVAL, "instance %d: NULL plan or vector", i);
    if (b[i] == x[i]) return fail(SMR_EINVAL, "instance %d: b and x must be distinct", i);
  }
  smr_status st = check_distinct_plans(count, plans);
  if (st != SMR_OK) return st;
  BatchState &bst = batch_state();
  std::lock_guard<std::mutex> lock(bst.mu);
  return solve_batched_locked(bst, count, plans, b, x0, x, rtol, maxit, d_ws, infos, stream);
}

smr_status smr_solve_adjoint(const smr_plan *pl, const double *g, double *lam, double rtol, int32_t maxit,
                             smr_info *info, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (!g || !lam || g == lam) return fail(SMR_EINVAL, "g and lambda must be distinct non-NULL pointers");
  if (!(rtol > 0.0) || maxit < 0) return fail(SMR_EINVAL, "need rtol > 0 and maxit >= 0");
  const Plan &p = pl->p;
  hipStream_t s = (hipStream_t)stream;
  Ctx c{&p, s};
  // (Y T) mu = g  <=>  (Y T) mu = Y (Y g): solve with b' = Y g, then lambda = Y mu
  LAUNCH(PROF_VEC, launch_scale_copy(c, g, p.G, 1.0, 1));
  st = use_spectral(p) ? minres_spectral(p, s, p.G, nullptr, lam, rtol, maxit, info)
                       : minres(p, s, p.G, nullptr, lam, rtol, maxit, info);
  if (st != SMR_OK && st != SMR_ENOTCONV) return st;
  LAUNCH(PROF_VEC, launch_scale_copy(c, lam, p.G, 1.0, 1));
  HIP_TRY(hipMemcpyAsync(lam, p.G, p.len * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return st;
}

smr_status smr_solve_adjoint_batched(int32_t count, const smr_plan *const *plans, const double *const *g,
                                     double *const *lam, double rtol, int32_t maxit, void *d_ws, size_t ws_bytes,
                                     smr_info *infos, void *stream) {
  if (count < 0 || (count > 0 && (!plans || !g || !lam || !infos))) return fail(SMR_EINVAL, "bad batch arguments");
  for (int i = 0; i < count; ++i)
    if (!plans[i]) return fail(SMR_EINVAL, "instance %d: NULL plan", i);
  smr_status st0 = check_distinct_plans(count, plans);
  if (st0 != SMR_OK) return st0;
  hipStream_t s = (hipStream_t)stream;
  std::vector<const double *> bs(count);
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !g[i] || !lam[i] || g[i] == lam[i]) return fail(SMR_EINVAL, "instance %d: bad pointers", i);
    const Plan &p = plans[i]->p;
    Ctx c{&p, s};
    LAUNCH(PROF_VEC, launch_scale_copy(c, g[i], p.G, 1.0, 1));   // (Y T) mu = g  <=>  solve with b' = Y g
    bs[i] = p.G;
  }
  smr_status st =
      smr_minres_solve_batched(count, plans, bs.data(), nullptr, lam, rtol, maxit, d_ws, ws_bytes, infos, stream);
  if (st != SMR_OK && st != SMR_ENOTCONV) return st;
  for (int i = 0; i < count; ++i) {                           // lambda = Y mu
    const Plan &p = plans[i]->p;
    Ctx c{&p, s};
    LAUNCH(PROF_VEC, launch_scale_copy(c, lam[i], p.G, 1.0, 1));
    HIP_TRY(hipMemcpyAsync(lam[i], p.G, p.len * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return st;
}

smr_status smr_rhs_adjoint(const smr_plan *pl, const double *lam, double *gf, double *gu0, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (pl->p.scheme != SMR_THETA) return fail(SMR_EINVAL, "smr_rhs_adjoint is defined for the theta scheme");
  if (!lam || !gf) return fail(SMR_EINVAL, "lambda and grad_f must be non-NULL");
  Ctx c{&pl->p, (hipStream_t)stream};
  LAUNCH(PROF_STENCIL, launch_rhs_adjoint(c, lam, gf, gu0));
  return SMR_OK;
}

smr_status smr_grad_a(const smr_plan *pl, const double *u, const double *u0, const double *lam, double *gax,
                      double *gay, double *gnodal, void *stream) {
  smr_status st = check_plan(pl);
  if (st != SMR_OK) return st;
  if (!u || !lam) return fail(SMR_EINVAL, "u and lambda must be non-NULL");
  const Plan &p = pl->p;
  if (p.dim == 3) return fail(SMR_EUNSUPPORTED, "the coefficient gradient is implemented for dim 1 and 2");
  double *fx = gax ? gax : p.gface;
  double *fy = p.dim == 1 ? nullptr : (gay ? gay : p.gface + (size_t)p.N * (p.N + 1));
  Ctx c{&p, (hipStream_t)stream};
  LAUNCH(PROF_STENCIL, launch_grad_faces(c, u, u0, lam, fx, fy, gnodal));
  return SMR_OK;
}

}  // extern "C"

extern "C" {

smr_status smr_profile_enable(int32_t on) {
  if (on) {
    g_prof.clear();
    g_prof.on = true;
  } else {
    g_prof.on = false;
  }
  return SMR_OK;
}

smr_status smr_profile_read(int32_t cls, int32_t *launches, double *total_ms) {
  if (cls < 0 || cls >= PROF_NCLASS || !launches || !total_ms) return fail(SMR_EINVAL, "bad profile query");
  double tot = 0.0;
  long n = 0;
  for (auto &pr : g_prof.rec[cls]) {
    HIP_TRY(hipEventSynchronize(pr.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.a, pr.b));
    tot += ms;
    n += pr.count;
  }
  *launches = (int32_t)n;
  *total_ms = tot;
  return SMR_OK;
}

}  // extern "C"
