"""ctypes binding of the C ABI declared in include/smr.h.

Argument marshalling only: every step of the solve runs in the HIP kernels of
libsmr.so.  PyTorch supplies device memory (the plan workspace and the vectors) and
the current HIP stream.  If libsmr.so is missing the import-time loader raises; there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmr.so")

SMR_OK, SMR_EINVAL, SMR_EWORKSPACE, SMR_EDEVICE, SMR_ENOTSPD, SMR_EBREAKDOWN, SMR_ENOTCONV, SMR_EUNSUPPORTED = range(8)
STATUS_NAMES = {0: "ok", 1: "einval", 2: "eworkspace", 3: "edevice", 4: "enotspd", 5: "ebreakdown",
                6: "enotconv", 7: "eunsupported"}
SCHEMES = {"theta": 0, "bdf2": 2, "bdf3": 3, "bdf4": 4}
PRECONDS = {"PH": 0, "PTHETA_CHEB": 2, "NONE": 3}
PPRECS = {"fp64": 0, "fp32": 1, "bf16": 2}

# Every entry point of include/smr.h.
EXPORTS = (
    "smr_workspace_size", "smr_setup", "smr_destroy", "smr_build_rhs", "smr_apply_A", "smr_apply_P_inv",
    "smr_minres_solve", "smr_batch_workspace_size", "smr_minres_solve_batched", "smr_solve_adjoint", "smr_solve_adjoint_batched", "smr_rhs_adjoint", "smr_grad_a",
    "smr_profile_enable", "smr_profile_read", "smr_version", "smr_last_error", "smr_tile_cols",
    "smr_apply_P_inv_static", "smr_pinv_variant", "smr_tune_stats", "smr_tune_reset", "smr_matvec_tiles",
)
STATIC_SCRATCH_BYTES = 64 << 20   # SMR_STATIC_SCRATCH_BYTES
PROFILE_CLASSES = {"time": 0, "dst": 1, "stencil": 2, "vec": 3, "scalar": 4, "spec": 5, "kslice": 6}


class SmrDesc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("N", ctypes.c_int32), ("n", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("precond", ctypes.c_int32), ("pprec", ctypes.c_int32), ("cheb_k", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("T", ctypes.c_double), ("theta", ctypes.c_double),
        ("ax_host", ctypes.c_void_p), ("ay_host", ctypes.c_void_p), ("a_nodal_host", ctypes.c_void_p),
        ("az_host", ctypes.c_void_p),
    ]


class SmrInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres_true", ctypes.c_double), ("relres_prec", ctypes.c_double),
                ("res_evals", ctypes.c_int32), ("tile_cols", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "status": STATUS_NAMES.get(self.status, self.status),
                "relres_true": self.relres_true, "relres_prec": self.relres_prec,
                "res_evals": self.res_evals, "tile_cols": self.tile_cols}


class SmrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libsmr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2201_10062_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.smr_workspace_size.argtypes = [ctypes.POINTER(SmrDesc), ctypes.POINTER(ctypes.c_size_t)]
    lib.smr_setup.argtypes = [ctypes.POINTER(SmrDesc), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.smr_destroy.argtypes = [P]
    lib.smr_tile_cols.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.smr_pinv_variant.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.smr_matvec_tiles.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    lib.smr_tune_stats.argtypes = [ctypes.POINTER(ctypes.c_int64)] * 3
    lib.smr_tune_reset.argtypes = []
    lib.smr_build_rhs.argtypes = [P, P, P, P, P]
    lib.smr_apply_A.argtypes = [P, P, P, P]
    lib.smr_apply_P_inv.argtypes = [P, P, P, P]
    lib.smr_apply_P_inv_static.argtypes = [P, P, P, P]
    lib.smr_minres_solve.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(SmrInfo), P]
    lib.smr_batch_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)]
    lib.smr_minres_solve_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P),
                                             ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_double,
                                             ctypes.c_int32, P, ctypes.c_size_t, ctypes.POINTER(SmrInfo), P]
    lib.smr_solve_adjoint.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(SmrInfo), P]
    lib.smr_solve_adjoint_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P),
                                              ctypes.POINTER(P), ctypes.c_double, ctypes.c_int32, P,
                                              ctypes.c_size_t, ctypes.POINTER(SmrInfo), P]
    lib.smr_rhs_adjoint.argtypes = [P, P, P, P, P]
    lib.smr_grad_a.argtypes = [P, P, P, P, P, P, P, P]
    lib.smr_profile_enable.argtypes = [ctypes.c_int32]
    lib.smr_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.smr_version.restype = ctypes.c_char_p
    lib.smr_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("smr_version", "smr_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int):
    if st != SMR_OK:
        raise SmrError(st, load().smr_last_error().decode())


FLAG_GENERAL_PATH = 1
FLAG_TILE16 = 2
FLAG_TILE32 = 4
FLAG_TILE64 = 128
PINV_FLAGS = {None: 0, "f64": 8, "f32": 16, "f32c16": 32, "f64c16": 64}
MATVEC_FLAGS = {None: 0, "level": 256, "tiles": 512}


def make_desc(dim, N, n, scheme="theta", theta=1.0, T=1.0, precond="PH", pprec="fp64", cheb_k=3,
              ax=None, ay=None, a_nodal=None, general_path=False, tile_cols=None, az=None, pinv=None, matvec=None):
    """Build an SmrDesc; returns (desc, keepalive) where keepalive holds the host arrays.
    tile_cols: None (timed at setup), 16, 32 or 64 (ceil(n/2) <= 64, or 128 with pprec="fp32").  pinv: None (timed at setup), "f64", "f64c16",
    "f32" or "f32c16" (the physical-basis P^{-1} variant; the float32 ones for float32 plans).
    matvec: None (timed at setup), "level" or "tiles" (form of the N = 127 per-level matvec)."""
    if tile_cols not in (None, 16, 32, 64):
        raise ValueError(f"tile_cols must be None, 16, 32 or 64 (got {tile_cols})")
    if pinv not in PINV_FLAGS:
        raise ValueError(f"pinv must be one of {list(PINV_FLAGS)} (got {pinv})")
    if matvec not in MATVEC_FLAGS:
        raise ValueError(f"matvec must be one of {list(MATVEC_FLAGS)} (got {matvec})")
    keep = []

    def host(a):
        if a is None:
            return None
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        keep.append(arr)
        return arr.ctypes.data

    d = SmrDesc(dim=dim, N=N, n=n, scheme=SCHEMES[scheme], precond=PRECONDS[precond], pprec=PPRECS[pprec],
                cheb_k=cheb_k, flags=(FLAG_GENERAL_PATH if general_path else 0)
                | {None: 0, 16: FLAG_TILE16, 32: FLAG_TILE32, 64: FLAG_TILE64}[tile_cols] | PINV_FLAGS[pinv]
                | MATVEC_FLAGS[matvec], T=T, theta=theta,
                ax_host=host(ax), ay_host=host(ay), a_nodal_host=host(a_nodal), az_host=host(az))
    return d, keep


def profile_enable(on: bool = True):
    """Start (clearing old records) or stop event timing of every kernel launch."""
    _check(load().smr_profile_enable(1 if on else 0))


def profile_read(cls: str):
    """(launches, total_ms) recorded for one kernel class since profile_enable(True)."""
    n = ctypes.c_int32(0)
    ms = ctypes.c_double(0.0)
    _check(load().smr_profile_read(PROFILE_CLASSES[cls], ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def tune_stats():
    """(entries, hits, misses) of the autotuner's process-wide cache."""
    v = [ctypes.c_int64(0) for _ in range(3)]
    _check(load().smr_tune_stats(*[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def tune_reset():
    """Clear the autotuner's cache: the next plans and batches time their choices again."""
    _check(load().smr_tune_reset())


def workspace_size(**kw) -> int:
    d, _keep = make_desc(**kw)
    out = ctypes.c_size_t(0)
    _check(load().smr_workspace_size(ctypes.byref(d), ctypes.byref(out)))
    return out.value


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A solver plan on the current device; owns its workspace (a torch uint8 tensor)."""

    def __init__(self, dim: int, N: int, n: int, scheme: str = "theta", theta: float = 1.0, T: float = 1.0,
                 precond: str = "PH", pprec: str = "fp64", cheb_k: int = 3, ax=None, ay=None, a_nodal=None,
                 device="cuda", general_path: bool = False, tile_cols=None, workspace=None, az=None, pinv=None,
                 matvec=None):
        """ax, ay, az: face values (az with dim 3 only); a_nodal: nodal values (dim 1, 2).
        workspace: a uint8 device tensor to build the plan in (e.g. the ``raw_workspace``
        of a plan that is no longer used); a new one is allocated when it is None or too small."""
        import torch
        self.lib = load()
        self.dim, self.N, self.n = dim, N, n
        self.m = N ** dim
        self.scheme, self.theta, self.T = scheme, float(theta), float(T)
        self.precond, self.pprec = precond, pprec
        self.device = torch.device(device)
        d, keep = make_desc(dim, N, n, scheme, theta, T, precond, pprec, cheb_k, ax, ay, a_nodal, general_path,
                            tile_cols, az, pinv, matvec)
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.smr_workspace_size(ctypes.byref(d), ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        raw = workspace
        if raw is None or raw.device != self.device or raw.dtype != torch.uint8 or \
                raw.numel() < self.ws_bytes + (-raw.data_ptr()) % 256:
            raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + self.ws_bytes]
        h = ctypes.c_void_p(0)
        _check(self.lib.smr_setup(ctypes.byref(d), ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                  _stream(), ctypes.byref(h)))
        self.handle = h
        del keep

    @property
    def tile_cols(self) -> int:
        """Column-tile width of the sine-basis solve (16, 32 or 64), 0 on the physical-basis path."""
        c = ctypes.c_int32(0)
        _check(self.lib.smr_tile_cols(self.handle, ctypes.byref(c)))
        return c.value

    @property
    def pinv_variant(self) -> str:
        """The physical-basis P^{-1} variant ("f64", "f64c16", "f32", "f32c16"), or None
        (sine-basis solves, P = I)."""
        c = ctypes.c_int32(0)
        _check(self.lib.smr_pinv_variant(self.handle, ctypes.byref(c)))
        return {0: "f64", 1: "f32", 2: "f32c16", 3: "f64c16"}.get(c.value)

    @property
    def matvec_tiles(self) -> bool:
        """True when the per-level matvec runs as tiled passes (N = 127, variable a, sine basis)."""
        c = ctypes.c_int32(0)
        _check(self.lib.smr_matvec_tiles(self.handle, ctypes.byref(c)))
        return c.value == 1

    @property
    def raw_workspace(self):
        """The device tensor holding the workspace (reusable by a later plan once this one is
        released)."""
        return self._raw

    def release(self):
        """Destroy the host-side plan now (its workspace tensor stays valid for reuse)."""
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.smr_destroy(h)
        self.handle = None

    def __del__(self):
        self.release()

    # --- helpers
    def _vec(self, t, n_levels=None):
        import torch
        n_levels = self.n if n_levels is None else n_levels
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.ws.device or t.numel() != n_levels * self.m:
            raise ValueError(f"expected a contiguous float64 tensor of {n_levels * self.m} elements on {self.ws.device}")
        return t

    def empty(self, levels=None):
        import torch
        return torch.empty((self.n if levels is None else levels) * self.m, dtype=torch.float64, device=self.ws.device)

    # --- entry points
    def build_rhs(self, f, u0=None, out=None):
        self._vec(f, self.n + 1)
        b = self.empty() if out is None else self._vec(out)
        _check(self.lib.smr_build_rhs(self.handle, _ptr(f), _ptr(u0), _ptr(b), _stream()))
        return b

    def apply_A(self, x, out=None):
        self._vec(x)
        y = self.empty() if out is None else self._vec(out)
        _check(self.lib.smr_apply_A(self.handle, _ptr(x), _ptr(y), _stream()))
        return y

    def apply_P_inv(self, v, out=None):
        self._vec(v)
        z = self.empty() if out is None else self._vec(out)
        _check(self.lib.smr_apply_P_inv(self.handle, _ptr(v), _ptr(z), _stream()))
        return z

    def apply_P_inv_static(self, v, out=None):
        """P^{-1} v with the intermediate vectors in the library's static device scratch
        (allocates nothing in the library; calls overlapping on one GPU race)."""
        self._vec(v)
        z = self.empty() if out is None else self._vec(out)
        _check(self.lib.smr_apply_P_inv_static(self.handle, _ptr(v), _ptr(z), _stream()))
        return z

    def solve(self, b, x0=None, rtol=1e-8, maxit=500, raise_on_fail=True):
        """MINRES on Y T x = Y b from x0 (None: x0 = 0); returns (x, info dict)."""
        self._vec(b)
        if x0 is not None:
            self._vec(x0)
        x = self.empty()
        info = SmrInfo()
        st = self.lib.smr_minres_solve(self.handle, _ptr(b), _ptr(x0), _ptr(x), float(rtol), int(maxit),
                                       ctypes.byref(info), _stream())
        if st != SMR_OK and raise_on_fail and st != SMR_ENOTCONV:
            _check(st)
        return x, info.as_dict()

    def solve_adjoint(self, g, rtol=1e-8, maxit=500):
        self._vec(g)
        lam = self.empty()
        info = SmrInfo()
        st = self.lib.smr_solve_adjoint(self.handle, _ptr(g), _ptr(lam), float(rtol), int(maxit),
                                        ctypes.byref(info), _stream())
        if st not in (SMR_OK, SMR_ENOTCONV):
            _check(st)
        return lam, info.as_dict()

    def rhs_adjoint(self, lam, want_u0=True):
        self._vec(lam)
        gf = self.empty(self.n + 1)
        gu0 = self.empty(1) if want_u0 else None
        _check(self.lib.smr_rhs_adjoint(self.handle, _ptr(lam), _ptr(gf), _ptr(gu0), _stream()))
        return gf, gu0

    def grad_a(self, u, lam, u0=None):
        import torch
        self._vec(u)
        self._vec(lam)
        N, dim = self.N, self.dim
        dev = self.ws.device
        gax = torch.empty(N + 1 if dim == 1 else N * (N + 1), dtype=torch.float64, device=dev)
        gay = None if dim == 1 else torch.empty((N + 1) * N, dtype=torch.float64, device=dev)
        gn = torch.empty((N + 2) ** dim, dtype=torch.float64, device=dev)
        _check(self.lib.smr_grad_a(self.handle, _ptr(u), _ptr(u0), _ptr(lam), _ptr(gax), _ptr(gay), _ptr(gn),
                                   _stream()))
        return gax, gay, gn


class Batch:
    """A fixed set of plans solved together; owns the batch workspace (descriptor table)."""

    def __init__(self, plans: Sequence[Plan], workspace=None):
        """workspace: a uint8 device tensor to reuse (e.g. ``raw_workspace`` of an earlier
        batch of the same plan layout, whose captured iterations are then replayed)."""
        import torch
        self.plans = list(plans)
        n = len(self.plans)
        P = ctypes.c_void_p
        self._hp = (P * n)(*[p.handle.value for p in self.plans])
        nbytes = ctypes.c_size_t(0)
        _check(load().smr_batch_workspace_size(n, self._hp, ctypes.byref(nbytes)))
        dev = self.plans[0].ws.device if n else torch.device("cuda")
        raw = workspace
        if raw is None or raw.device != dev or raw.dtype != torch.uint8 or \
                raw.numel() < nbytes.value + (-raw.data_ptr()) % 256:
            raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + nbytes.value]

    @property
    def raw_workspace(self):
        return self._raw

    def solve(self, bs, x0s=None, rtol=1e-8, maxit=500):
        """Solve every (plan, b) pair from x0s (None: every x0 = 0); returns (xs, infos)."""
        n = len(self.plans)
        xs = [p.empty() for p in self.plans]
        for p, b in zip(self.plans, bs):
            p._vec(b)
        P = ctypes.c_void_p
        x0p = None
        if x0s is not None:
            for p, x0 in zip(self.plans, x0s):
                if x0 is not None:
                    p._vec(x0)
            x0p = (P * n)(*[_ptr(x0) for x0 in x0s])
        bp = (P * n)(*[b.data_ptr() for b in bs])
        xp = (P * n)(*[x.data_ptr() for x in xs])
        infos = (SmrInfo * n)()
        st = load().smr_minres_solve_batched(n, self._hp, bp, x0p, xp, float(rtol), int(maxit),
                                             ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), infos, _stream())
        if st not in (SMR_OK, SMR_ENOTCONV):
            _check(st)
        return xs, [i.as_dict() for i in infos]


    def solve_adjoint(self, gs, rtol=1e-8, maxit=500):
        """Solve T_i^T lambda_i = g_i for every plan; returns (lambdas, infos)."""
        n = len(self.plans)
        lams = [p.empty() for p in self.plans]
        for p, g in zip(self.plans, gs):
            p._vec(g)
        P = ctypes.c_void_p
        gp = (P * n)(*[g.data_ptr() for g in gs])
        lp = (P * n)(*[x.data_ptr() for x in lams])
        infos = (SmrInfo * n)()
        st = load().smr_solve_adjoint_batched(n, self._hp, gp, lp, float(rtol), int(maxit),
                                              ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), infos, _stream())
        if st not in (SMR_OK, SMR_ENOTCONV):
            _check(st)
        return lams, [i.as_dict() for i in infos]


def solve_batched(plans: Sequence[Plan], bs, rtol=1e-8, maxit=500):
    """Solve every (plan, b) pair in one batched call; returns (xs, infos)."""
    return Batch(plans).solve(bs, rtol=rtol, maxit=maxit)
