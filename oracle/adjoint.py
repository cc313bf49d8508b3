"""Adjoint solve and gradients (oracle; test infrastructure only).

Because Y T is symmetric and Y^2 = I, T^T = Y T Y (eqn:main_system), so
T^T lambda = g is (Y T)(Y lambda) = g: the same preconditioned MINRES with
right-hand side g, followed by a flip.

For the theta scheme write the residual of every time level k = 1..n as
R_k = u_k - u_{k-1} + tau K(a)(theta u_k + (1-theta) u_{k-1}) - tau(theta f^k + (1-theta) f^{k-1})
with u_0 = u0 (this is T u - f_H of Sec. 1 with the u0 term moved into R_1).
For a loss L(u) with g = dL/du and T^T lambda = g:
  dL/df^k  = theta tau lambda_k + (1-theta) tau lambda_{k+1}   (lambda_0 = lambda_{n+1} = 0)
  dL/du0   = (I - (1-theta) tau K) lambda_1
  dL/da_e  = -(tau/h^2) sum_k (D_e lambda_k)(D_e utilde_k),  utilde_k = theta u_k + (1-theta) u_{k-1}
where K(a) = sum_e a_e D_e^T D_e / h^2 and D_e is the difference across face e.
A nodal coefficient enters through face = mean of its two nodes, so the nodal
gradient is half the sum of the gradients of the faces touching the node.
"""
from __future__ import annotations

import numpy as np

from . import spatial


def adjoint_solve(system, g: np.ndarray, rtol: float = 1e-8, maxit: int = 500):
    """lambda with T^T lambda = g, via MINRES on (Y T) mu = g and lambda = Y mu."""
    from .minres import minres
    res = minres(system.apply_YT, system.apply_Pinv, np.asarray(g, dtype=np.float64), rtol=rtol, maxit=maxit)
    return system.flip(res.x), res


def adjoint_direct(system, g: np.ndarray) -> np.ndarray:
    """T^T lambda = g by backward block substitution: T^T is block upper-banded with A_l^T = A_l
    (K symmetric) on the l-th block superdiagonal, one sparse SPD solve per level."""
    import scipy.sparse.linalg as spla
    n = system.n
    G = np.asarray(g, dtype=np.float64).reshape(n, -1)
    lu = spla.splu(system.blocks[0].tocsc())
    L = np.zeros_like(G)
    for k in range(n - 1, -1, -1):
        r = G[k].copy()
        for l in range(1, len(system.blocks)):
            if k + l < n:
                r -= system.blocks[l].T @ L[k + l]
        L[k] = lu.solve(r)
    return L.reshape(-1)


def adjoint_dense(system, g: np.ndarray) -> np.ndarray:
    T = system.assemble_T().toarray()
    return np.linalg.solve(T.T, g)


def rhs_adjoint(system, lam: np.ndarray):
    """(dL/df of shape (n+1, m), dL/du0 of shape (m,)) for the theta scheme."""
    n, m, tau, th = system.n, system.m, system.tau, system.theta
    L = np.asarray(lam).reshape(n, m)
    gf = np.zeros((n + 1, m))
    gf[1:] += th * tau * L
    gf[:-1] += (1.0 - th) * tau * L
    gu0 = L[0] - (1.0 - th) * tau * (system.K @ L[0])
    return gf, gu0


def grad_faces(system, u: np.ndarray, u0: np.ndarray, lam: np.ndarray):
    """dL/da at the faces: (gax, gay) shaped like (ax, ay)."""
    n, m, tau, th, N, dim = system.n, system.m, system.tau, system.theta, system.N, system.dim
    U = np.asarray(u).reshape(n, m)
    Uprev = np.vstack([np.asarray(u0, dtype=np.float64).reshape(1, m), U[:-1]])
    if system.scheme == "theta":
        Ut = th * U + (1.0 - th) * Uprev
    else:
        Ut = U
    L = np.asarray(lam).reshape(n, m)
    Dx, Dy = spatial.face_difference(N, dim)
    h2 = system.h ** 2
    gx = -(tau / h2) * np.sum((Dx @ L.T) * (Dx @ Ut.T), axis=1)
    if dim == 1:
        return gx, None
    gy = -(tau / h2) * np.sum((Dy @ L.T) * (Dy @ Ut.T), axis=1)
    return gx.reshape(N, N + 1), gy.reshape(N + 1, N)


def grad_nodal(gx: np.ndarray, gy, N: int, dim: int) -> np.ndarray:
    if dim == 1:
        g = np.zeros(N + 2)
        g[:-1] += 0.5 * gx
        g[1:] += 0.5 * gx
        return g
    g = np.zeros((N + 2, N + 2))
    g[1:-1, :-1] += 0.5 * gx
    g[1:-1, 1:] += 0.5 * gx
    g[:-1, 1:-1] += 0.5 * gy
    g[1:, 1:-1] += 0.5 * gy
    return g
