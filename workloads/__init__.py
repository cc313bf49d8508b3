"""Seeded synthetic inputs for all-at-once heat-equation solves.

This module only samples the PDE data (coefficient a, source f, initial value u0,
right-hand sides) on the finite-difference grid and draws seeded random numbers.
It contains none of the solver's arithmetic: no stiffness matrix, no time
discretisation, no transform, no preconditioner, no Krylov step.  Both the FP64
CPU oracle's tests and the GPU path consume exactly these arrays.

Grid convention (finite differences on the unit interval / unit square, as in the
numerical section of Hon, Fung, Dong, Serra-Capizzano, arXiv 2201.10062):
  h = 1/(N+1), interior nodes x_i = i*h, i = 1..N, time levels t_k = k*tau,
  tau = T/n, k = 0..n.  Arrays are C-ordered (time, y, x) with x fastest.
Face coefficients (the a_{j+1/2} of the variable-coefficient stiffness matrix,
Sec. 3.1.1): in 1D ``ax[i]`` is a((i+1/2)h), i = 0..N.  In 2D ``ax[j, i]`` is
a((i+1/2)h, (j+1)h) (shape N x (N+1)) and ``ay[j, i]`` is a((i+1)h, (j+1/2)h)
(shape (N+1) x N).  Nodal coefficients cover the (N+2)^dim grid including the
boundary nodes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

__all__ = [
    "Problem", "interior", "sample_faces", "sample_nodal", "sample_grid_fn",
    "manufactured_1d", "crank_nicolson_2d_noisy", "variable_coef_2d",
    "bdf2_batch", "inverse_problem_2d", "example1", "example2", "example2_exact",
    "bdf2_batch_spec", "bump_centres", "example3",
]


@dataclasses.dataclass
class Problem:
    """One all-at-once heat-equation instance.

    scheme: "theta" (two-level theta-method) or "bdf2".
    f: (n+1, N^dim) source samples at t_0..t_n (theta scheme), or None.
    b: (n, N^dim) right-hand side given directly (BDF2 batch), or None.
    u0: (N^dim,) initial value at interior nodes.
    ax, ay, az: face coefficients (None means a == 1 everywhere; az in 3D only).
    a_nodal: nodal coefficient on the (N+2)^dim grid, or None.
    """
    dim: int
    N: int
    n: int
    T: float = 1.0
    scheme: str = "theta"
    theta: float = 1.0
    f: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None
    u0: Optional[np.ndarray] = None
    ax: Optional[np.ndarray] = None
    ay: Optional[np.ndarray] = None
    a_nodal: Optional[np.ndarray] = None
    name: str = ""
    az: Optional[np.ndarray] = None

    @property
    def m(self) -> int:
        return self.N ** self.dim

    @property
    def tau(self) -> float:
        return self.T / self.n

    @property
    def h(self) -> float:
        return 1.0 / (self.N + 1)

    @property
    def const_coef(self) -> bool:
        return self.ax is None


def interior(N: int) -> np.ndarray:
    return np.arange(1, N + 1, dtype=np.float64) / (N + 1)


def sample_faces(a: Callable, N: int, dim: int):
    """Sample a(x[, y]) at the face midpoints used by the 3/5-point stencil."""
    h = 1.0 / (N + 1)
    half = (np.arange(N + 1, dtype=np.float64) + 0.5) * h
    xi = interior(N)
    if dim == 1:
        return np.asarray(a(half), dtype=np.float64).copy(), None
    X, Y = np.meshgrid(half, xi, indexing="xy")        # shape (N, N+1): rows y_j
    ax = np.asarray(a(X, Y), dtype=np.float64)
    X, Y = np.meshgrid(xi, half, indexing="xy")        # shape (N+1, N)
    ay = np.asarray(a(X, Y), dtype=np.float64)
    return np.ascontiguousarray(ax), np.ascontiguousarray(ay)


def sample_nodal(a: Callable, N: int, dim: int) -> np.ndarray:
    """Sample a on the (N+2)^dim nodes including the boundary."""
    g = np.arange(N + 2, dtype=np.float64) / (N + 1)
    if dim == 1:
        return np.asarray(a(g), dtype=np.float64).copy()
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.ascontiguousarray(np.asarray(a(X, Y), dtype=np.float64))


def sample_grid_fn(fn: Callable, N: int, dim: int, times: np.ndarray) -> np.ndarray:
    """Sample fn(x[, y], t) at interior nodes for each time in ``times``.

    Returns shape (len(times), N^dim), x fastest."""
    xi = interior(N)
    out = []
    for t in times:
        if dim == 1:
            out.append(np.asarray(fn(xi, t), dtype=np.float64) * np.ones(N))
        else:
            X, Y = np.meshgrid(xi, xi, indexing="xy")
            out.append((np.asarray(fn(X, Y, t), dtype=np.float64) * np.ones((N, N))).reshape(-1))
    return np.ascontiguousarray(np.stack(out))


def _times(n: int, T: float) -> np.ndarray:
    return np.arange(n + 1, dtype=np.float64) * (T / n)


# --------------------------------------------------------------------------
# The five workloads (all synthetic; the paper's own examples are analytic).
# --------------------------------------------------------------------------

def manufactured_1d(N: int = 63, n: int = 64, theta: float = 1.0) -> Problem:
    """1D, a = 1, exact u = sin(pi x) e^t, so f = (1 + pi^2) sin(pi x) e^t, g = 0."""
    pi = math.pi
    f = sample_grid_fn(lambda x, t: (1 + pi * pi) * np.sin(pi * x) * math.exp(t), N, 1, _times(n, 1.0))
    u0 = np.sin(pi * interior(N))
    return Problem(dim=1, N=N, n=n, theta=theta, f=f, u0=u0, name=f"manufactured_1d_N{N}_n{n}")


def crank_nicolson_2d_noisy(N: int = 127, n: int = 256, seed: int = 0, noise: float = 1e-3,
                            theta: float = 0.5) -> Problem:
    """2D, a = 1, u = sin(pi x) sin(pi y) e^{-t} gives f = (2 pi^2 - 1) u; plus iid
    N(0, noise^2) per interior node and time level k = 0..n from default_rng(seed)."""
    pi = math.pi
    f = sample_grid_fn(lambda x, y, t: (2 * pi * pi - 1) * np.sin(pi * x) * np.sin(pi * y) * math.exp(-t),
                       N, 2, _times(n, 1.0))
    if noise:
        rng = np.random.default_rng(seed)
        f = f + noise * rng.standard_normal((n + 1, N, N)).reshape(n + 1, N * N)
    xi = interior(N)
    X, Y = np.meshgrid(xi, xi, indexing="xy")
    u0 = (np.sin(pi * X) * np.sin(pi * Y)).reshape(-1)
    return Problem(dim=2, N=N, n=n, theta=theta, f=np.ascontiguousarray(f), u0=u0,
                   name=f"cn2d_noisy_N{N}_n{n}")


def variable_coef_2d(N: int = 255, n: int = 512, seed: int = 1, theta: float = 1.0) -> Problem:
    """2D, a = 1 + 0.5 sin(2 pi x) sin(2 pi y) at faces, f ~ U(-1, 1) from default_rng(seed)."""
    pi = math.pi
    ax, ay = sample_faces(lambda x, y: 1.0 + 0.5 * np.sin(2 * pi * x) * np.sin(2 * pi * y), N, 2)
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1.0, 1.0, size=(n + 1, N, N)).reshape(n + 1, N * N)
    return Problem(dim=2, N=N, n=n, theta=theta, f=np.ascontiguousarray(f), u0=np.zeros(N * N),
                   ax=ax, ay=ay, name=f"varcoef2d_N{N}_n{n}")


def bdf2_batch_spec(count: int = 64, Ns=(31, 63, 127), ns=(64, 128, 256)):
    """(N, n, variable-coefficient?) for each instance of the BDF2 batch."""
    spec = []
    for i in range(count):
        spec.append((Ns[i % len(Ns)], ns[(i // len(Ns)) % len(ns)], (i // (len(Ns) * len(ns))) % 2 == 1))
    return spec


def bdf2_batch(count: int = 64, seed: int = 2, Ns=(31, 63, 127), ns=(64, 128, 256)) -> list:
    """Batch of BDF2 instances with uneven (N, n); a = 1 or a = 1 + 0.5 cos(pi x);
    right-hand sides b_i ~ N(0, 1) drawn from one default_rng(seed) stream in instance order."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (N, n, var) in enumerate(bdf2_batch_spec(count, Ns, ns)):
        b = rng.standard_normal((n, N, N)).reshape(n, N * N)
        ax = ay = None
        if var:
            ax, ay = sample_faces(lambda x, y: 1.0 + 0.5 * np.cos(math.pi * x) + 0.0 * y, N, 2)
        out.append(Problem(dim=2, N=N, n=n, scheme="bdf2", b=np.ascontiguousarray(b), u0=np.zeros(N * N),
                           ax=ax, ay=ay, name=f"bdf2_{i}_N{N}_n{n}_{'var' if var else 'const'}"))
    return out


def bump_centres():
    c = (0.2, 0.4, 0.6, 0.8)
    return [(x, y) for y in c for x in c]


def inverse_problem_2d(N: int = 127, n: int = 256, batch: int = 16, width: float = 0.1):
    """Differentiable-solve workload: Gaussian-bump sources (constant in time),
    u0 = 0, nodal truth a = 1 + 0.3 x y and nodal evaluation point a = 1.

    Returns (problems at a = 1, a_truth_nodal)."""
    centres = bump_centres()[:batch]
    probs = []
    for (cx, cy) in centres:
        f = sample_grid_fn(lambda x, y, t: np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * width * width)),
                           N, 2, _times(n, 1.0))
        probs.append(Problem(dim=2, N=N, n=n, theta=1.0, f=f, u0=np.zeros(N * N),
                             a_nodal=np.ones((N + 2, N + 2)), name=f"bump_{cx}_{cy}"))
    a_truth = sample_nodal(lambda x, y: 1.0 + 0.3 * x * y, N, 2)
    return probs, a_truth


# --------------------------------------------------------------------------
# The paper's own numerical examples (analytic data, Sec. 5).
# --------------------------------------------------------------------------

def example1(N: int, n: int, theta: float) -> Problem:
    """Example 1: 2D, a = 1e-5, u0 = x(x-1)y(y-1), f = g = 0, T = 1."""
    xi = interior(N)
    X, Y = np.meshgrid(xi, xi, indexing="xy")
    u0 = (X * (X - 1) * Y * (Y - 1)).reshape(-1)
    ax = np.full((N, N + 1), 1e-5)
    ay = np.full((N + 1, N), 1e-5)
    return Problem(dim=2, N=N, n=n, theta=theta, f=np.zeros((n + 1, N * N)), u0=u0, ax=ax, ay=ay,
                   name=f"example1_N{N}_n{n}_theta{theta}")


def _ex2_f(x, y, t):
    e = math.exp(-t)
    s = np.sin(math.pi * x * y)
    c = np.cos(math.pi * x * y)
    return (e * x * (1 - x) * (2e-5 * s - y * (1 - y) - math.pi * 1e-5 * c * x * (1 - 2 * y))
            + e * y * (1 - y) * (2e-5 * s - math.pi * 1e-5 * c * y * (1 - 2 * x)))


def example2(N: int, n: int, theta: float) -> Problem:
    """Example 2: 2D, a = 1e-5 sin(pi x y) at faces, exact u = e^{-t} x(1-x) y(1-y)."""
    ax, ay = sample_faces(lambda x, y: 1e-5 * np.sin(math.pi * x * y), N, 2)
    f = sample_grid_fn(_ex2_f, N, 2, _times(n, 1.0))
    xi = interior(N)
    X, Y = np.meshgrid(xi, xi, indexing="xy")
    u0 = (X * (1 - X) * Y * (1 - Y)).reshape(-1)
    return Problem(dim=2, N=N, n=n, theta=theta, f=f, u0=u0, ax=ax, ay=ay,
                   name=f"example2_N{N}_n{n}_theta{theta}")


def example3(N: int, n: int, theta: float) -> Problem:
    """Example 3: 3D, a = 1e-3, u0 = x(x-1)y(y-1)z(z-1), f = g = 0, T = 1."""
    xi = interior(N)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")      # [k, j, i], x fastest
    u0 = (X * (X - 1) * Y * (Y - 1) * Z * (Z - 1)).reshape(-1)
    a = 1e-3
    return Problem(dim=3, N=N, n=n, theta=theta, f=np.zeros((n + 1, N ** 3)), u0=u0,
                   ax=np.full((N, N, N + 1), a), ay=np.full((N, N + 1, N), a), az=np.full((N + 1, N, N), a),
                   name=f"example3_N{N}_n{n}_theta{theta}")


def example2_exact(N: int, n: int) -> np.ndarray:
    """Exact solution of Example 2 at t_1..t_n on interior nodes, shape (n, N*N)."""
    return sample_grid_fn(lambda x, y, t: math.exp(-t) * x * (1 - x) * y * (1 - y), N, 2,
                          _times(n, 1.0))[1:]
