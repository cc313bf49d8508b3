"""Preconditioned MINRES (oracle; test infrastructure only).

The paper runs MATLAB's built-in MINRES with a zero initial guess and a stopping
tolerance on the relative residual (Sec. 5) and prints no listing.  This is the
Paige-Saunders method written from its derivation: a Lanczos process in the
P^{-1} inner product builds the tridiagonal matrix, whose QR factorisation by
Givens rotations is updated one column per step, and the iterate is advanced
along search directions w_j (the columns of Z_k R_k^{-1}).

Stopping reading: the paper says only "relative residual" with tolerance 1e-6.
This oracle stops at the first iteration whose TRUE relative residual
||rhs - A x_j||_2 / ||rhs||_2 is <= rtol, evaluating it after every iteration.
That reading reproduces the paper's printed iteration counts (Tables 1-3), while
stopping on the rotated P^{-1}-norm estimate |eta|/gamma_1 does not.  With
rhs = Y f_H, ||rhs - Y T x|| = ||f_H - T x|| because Y is a permutation.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class MinresResult:
    x: np.ndarray
    iters: int
    status: str              # "converged", "maxit", "breakdown", "exact"
    relres_true: float
    relres_prec: float
    eta_history: list


def minres(apply_A, apply_Pinv, rhs: np.ndarray, rtol: float = 1e-8, maxit: int = 500,
           x0: np.ndarray | None = None) -> MinresResult:
    """Solve A x = rhs (A symmetric, P SPD) from x0 (default 0)."""
    rhs = np.asarray(rhs, dtype=np.float64)
    bnorm = float(np.linalg.norm(rhs))
    x = np.zeros_like(rhs) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    if bnorm == 0.0:
        return MinresResult(np.zeros_like(rhs), 0, "exact", 0.0, 0.0, [])
    v = rhs - apply_A(x) if x0 is not None else rhs.copy()
    if float(np.linalg.norm(v)) / bnorm <= rtol:
        return MinresResult(x, 0, "converged", float(np.linalg.norm(v)) / bnorm, 0.0, [])
    z = apply_Pinv(v)
    g2 = float(np.dot(z, v))
    if not (g2 > 0.0) or not math.isfinite(g2):
        raise ValueError("preconditioner is not SPD on the initial residual")
    gamma = math.sqrt(g2)
    gamma1 = gamma
    gamma_old = 1.0
    v_old = np.zeros_like(rhs)
    w = np.zeros_like(rhs)
    w_old = np.zeros_like(rhs)
    c_old = c = 1.0
    s_old = s = 0.0
    eta = gamma
    hist = []
    relres = float(np.linalg.norm(v)) / bnorm
    for it in range(1, maxit + 1):
        zt = z / gamma
        q = apply_A(zt)
        delta = float(np.dot(q, zt))
        v_new = q - (delta / gamma) * v - (gamma / gamma_old) * v_old
        z_new = apply_Pinv(v_new)
        g2 = float(np.dot(z_new, v_new))
        if g2 < 0.0 or not math.isfinite(g2):
            raise ValueError("preconditioner is not SPD (gamma^2 < 0)")
        gamma_new = math.sqrt(g2)
        # QR of the Lanczos tridiagonal: apply the two previous rotations to the new column
        a0 = c * delta - c_old * s * gamma
        a1 = math.sqrt(a0 * a0 + gamma_new * gamma_new)
        a2 = s * delta + c_old * c * gamma
        a3 = s_old * gamma
        if a1 == 0.0:
            return MinresResult(x, it - 1, "breakdown", relres, abs(eta) / gamma1, hist)
        c_old, c = c, a0 / a1
        s_old, s = s, gamma_new / a1
        w_new = (zt - a3 * w_old - a2 * w) / a1
        x = x + (c * eta) * w_new
        eta = -s * eta
        hist.append(abs(eta) / gamma1)
        w_old, w = w, w_new
        v_old, v = v, v_new
        z = z_new
        gamma_old, gamma = gamma, gamma_new
        relres = float(np.linalg.norm(rhs - apply_A(x))) / bnorm
        if relres <= rtol:
            return MinresResult(x, it, "converged", relres, abs(eta) / gamma1, hist)
        if gamma_new == 0.0:
            relres = float(np.linalg.norm(rhs - apply_A(x))) / bnorm
            return MinresResult(x, it, "exact", relres, 0.0, hist)
    relres = float(np.linalg.norm(rhs - apply_A(x))) / bnorm
    return MinresResult(x, maxit, "maxit", relres, abs(eta) / gamma1, hist)
