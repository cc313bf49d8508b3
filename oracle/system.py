"""One all-at-once problem with its preconditioner (oracle; test infrastructure only).

Ties the pieces together: K(a) (eqn:matrix_Km_va), the blocks of T (eq. theta or
eqn:matrix_gen), the flip Y (eqn:main_system), the right-hand side f_H (Sec. 1)
and one of the preconditioners
  "PH"        P_H / Phat with K (constant a) or the averaged Kbar (variable a)
  "PTHETA"    P_theta with exact per-mode solves (theta scheme only)
  "PTHETA_CHEB" P_theta with k-step Chebyshev per-mode solves
  "NONE"      identity
and runs MINRES on Y T u = Y f_H.
"""
from __future__ import annotations

import numpy as np

from . import allatonce as aao
from . import precond as pc
from . import spatial
from .minres import minres


class System:
    def __init__(self, dim: int, N: int, n: int, scheme: str = "theta", theta: float = 1.0,
                 ax=None, ay=None, a_nodal=None, T: float = 1.0, precond: str = "PH",
                 cheb_k: int = 3, az=None):
        self.dim, self.N, self.n, self.scheme, self.theta = dim, N, n, scheme, float(theta)
        self.T = float(T)
        self.tau = self.T / n
        self.h = 1.0 / (N + 1)
        self.m = N ** dim
        if a_nodal is not None:
            if dim == 3:
                raise ValueError("3D coefficients are given as face values")
            ax, ay = spatial.faces_from_nodal(a_nodal, dim)
        self.const = ax is None
        if ax is None:
            faces = spatial.const_faces(N, dim)
            ax, ay = faces[0], faces[1]
            az = faces[2] if dim == 3 else None
        self.ax, self.ay, self.az = ax, ay, az
        self.K = spatial.stiffness(N, dim, ax, ay, az)
        if scheme == "theta":
            self.blocks = aao.theta_blocks(self.K, self.tau, self.theta)
        elif scheme == "bdf2":
            self.blocks = aao.bdf2_blocks(self.K, self.tau)
        elif scheme in ("bdf3", "bdf4"):
            self.alpha = aao.bdf_coefficients(int(scheme[3]))
            self.blocks = aao.bdf_blocks(self.K, self.tau, int(scheme[3]))
        else:
            raise ValueError(scheme)
        self.precond = precond
        self.cheb_k = cheb_k
        self.a_min, self.a_max = spatial.coef_bounds(N, dim, ax, ay, az)
        # eigenvalues used by P_H / Phat: those of K itself when a is constant, of the
        # averaged Kbar otherwise (the two coincide for constant face values)
        self.mu = spatial.mu_kbar(N, dim, ax, ay, az)
        if scheme == "theta":
            self.sigma = pc.sigma_theta(self.mu, n, self.tau, self.theta)
        elif scheme == "bdf2":
            self.sigma = pc.sigma_bdf2(self.mu, n, self.tau)
        else:
            self.sigma = pc.sigma_bdf(self.mu, n, self.tau, self.alpha)

    # ------------------------------------------------------------ operators
    def rhs(self, f=None, u0=None, b=None) -> np.ndarray:
        """Unpermuted f_H (theta scheme from f and u0) or the given b (BDF-l)."""
        if b is not None:
            return np.asarray(b, dtype=np.float64).reshape(-1).copy()
        u0 = np.zeros(self.m) if u0 is None else np.asarray(u0, dtype=np.float64)
        return aao.rhs_theta(f, u0, self.K, self.tau, self.theta)

    def apply_T(self, x):
        return aao.apply_T(self.blocks, x, self.n)

    def apply_YT(self, x):
        return aao.apply_YT(self.blocks, x, self.n)

    def apply_Pinv(self, v):
        if self.precond == "PH":
            return pc.pinv_spectral(v, self.sigma, self.n, self.N, self.dim)
        if self.precond == "PTHETA":
            return pc.pinv_ptheta_exact(v, self.K, self.n, self.tau, self.theta)
        if self.precond == "PTHETA_CHEB":
            return pc.pinv_ptheta_cheb(v, self.K, self.N, self.dim, self.n, self.tau, self.theta,
                                       self.cheb_k, self.a_min, self.a_max)
        if self.precond == "NONE":
            return np.asarray(v, dtype=np.float64).copy()
        raise ValueError(self.precond)

    def assemble_T(self):
        return aao.assemble_T(self.blocks, self.n)

    def flip(self, x):
        return aao.flip_vec(x, self.n)

    # ------------------------------------------------------------ solves
    def solve(self, fH: np.ndarray, rtol: float = 1e-8, maxit: int = 500, x0=None, **kw):
        """MINRES on Y T u = Y f_H (x0 = 0 unless given)."""
        return minres(self.apply_YT, self.apply_Pinv, self.flip(fH), rtol=rtol, maxit=maxit, x0=x0, **kw)

    def solve_direct(self, fH: np.ndarray) -> np.ndarray:
        """u* = T^{-1} f_H by sequential block substitution."""
        return aao.sequential(self.blocks, fH, self.n)
