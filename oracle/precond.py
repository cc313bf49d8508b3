"""Sine-transform preconditioners (oracle; test infrastructure only).

P_H (def:matrix_P, Sec. 3.1.1): P_H = sqrt(T_n[|g_theta|^2]) with
|g_theta|^2 = A0^2 + A1^2 + 2 A0 A1 cos x (eqn:symbol_p).  With K = U Lambda U^T,
P_H = (S_n (x) U) sqrt(I (x) (L0^2 + L1^2) + D_n (x) 2 L0 L1) (S_n (x) U)^T, so
P_H^{-1} v = three steps: transform, divide by sigma_{j,k} = |l0_k + l1_k e^{i phi_j}|,
transform back (S_n and U are symmetric orthogonal, U = S_N or S_N (x) S_N).
Variable a: K is replaced by the averaged Toeplitz Kbar in the preconditioner only.

Phat (def:matrix_P_gen, Sec. 4): sqrt(I (x) qbar0 + P_n (x) qbar1 + ... + P_n^l (x) qbarl)
for BDF-l, whose eigenvalues are |ghat(phi_j)| with ghat the symbol eqn:symbol_h_gen.

P_theta (def:matrix_mod_P, Sec. 3.1.4 "Modified Preconditioner"):
H (x) I + H_theta (x) tau K; in the time-sine basis it is block diagonal with
blocks eta_j I + tau zeta_j K, eta_j = 2 sin(phi_j/2),
zeta_j = sqrt(theta^2 + (1-theta)^2 + 2 theta (1-theta) cos phi_j).
The per-mode SPD solve is exact (sparse LU) or a fixed k-step Chebyshev iteration
preconditioned by the sine-diagonal eta_j I + tau zeta_j abar K_lap; the paper
leaves the inner solver open (it names multigrid as one option).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .sine import cos_phi, dst, dstn, dst_matrix, tridiag_half


def phi(n: int) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) * np.pi / (n + 1)


def sigma_theta(mu: np.ndarray, n: int, tau: float, theta: float) -> np.ndarray:
    """sigma_{j,k} = |l0 + l1 e^{i phi_j}|, l0 = 1 + theta tau mu_k, l1 = -1 + (1-theta) tau mu_k.
    Shape (n, len(mu))."""
    mu = np.asarray(mu, dtype=np.float64)
    l0 = 1.0 + theta * tau * mu
    l1 = -1.0 + (1.0 - theta) * tau * mu
    e = np.exp(1j * phi(n))[:, None]
    return np.abs(l0[None, :] + l1[None, :] * e)


def sigma_bdf2(mu: np.ndarray, n: int, tau: float) -> np.ndarray:
    """|ghat(phi_j)| for BDF2: |(1.5 + tau mu_k) - 2 e^{i phi_j} + 0.5 e^{2 i phi_j}|."""
    mu = np.asarray(mu, dtype=np.float64)
    e = np.exp(1j * phi(n))[:, None]
    return np.abs((1.5 + tau * mu)[None, :] - 2.0 * e + 0.5 * e * e)


def sigma_bdf(mu: np.ndarray, n: int, tau: float, alpha) -> np.ndarray:
    """|ghat(phi_j)| for BDF-l (eqn:symbol_h_gen evaluated on the spatial eigenvalue mu_k):
    |(alpha_0 + tau mu_k) + sum_{k >= 1} alpha_k e^{i k phi_j}|.  Shape (n, len(mu))."""
    mu = np.asarray(mu, dtype=np.float64)
    e = np.exp(1j * phi(n))[:, None]
    g = (alpha[0] + tau * mu)[None, :] + 0j
    for k in range(1, len(alpha)):
        g = g + alpha[k] * e ** k
    return np.abs(g)


def pinv_spectral(v: np.ndarray, sigma: np.ndarray, n: int, N: int, dim: int) -> np.ndarray:
    """The three-step P^{-1} v of Sec. 3.1.1: vt = (S_n (x) U^T) v; zt = vt / sigma;
    z = (S_n (x) U) zt, with every axis transformed by the orthonormal DST-I."""
    shape = (n,) + (N,) * dim
    axes = tuple(range(dim + 1))
    vt = dstn(np.asarray(v, dtype=np.float64).reshape(shape), axes)
    zt = vt / sigma.reshape(shape)
    return dstn(zt, axes).reshape(-1)


# ---------------------------------------------------------------- dense forms (pins)

def block_tridiag_sq(A0: np.ndarray, A1: np.ndarray, n: int) -> np.ndarray:
    """T_n[|g_theta|^2] of def:matrix_P: diagonal A0^2 + A1^2, off-diagonals A0 A1."""
    m = A0.shape[0]
    D = A0 @ A0 + A1 @ A1
    O = A0 @ A1
    out = np.zeros((n * m, n * m))
    for k in range(n):
        out[k * m:(k + 1) * m, k * m:(k + 1) * m] = D
        if k + 1 < n:
            out[k * m:(k + 1) * m, (k + 1) * m:(k + 2) * m] = O
            out[(k + 1) * m:(k + 2) * m, k * m:(k + 1) * m] = O
    return out


def sqrtm_spd(A: np.ndarray) -> np.ndarray:
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.sqrt(w)) @ V.T


def PH_dense(A0: np.ndarray, A1: np.ndarray, n: int) -> np.ndarray:
    return sqrtm_spd(block_tridiag_sq(A0, A1, n))


def Phat_dense(blocks, n: int) -> np.ndarray:
    """Phat for l = 2 by def:matrix_P_gen with qbar0 = q0 - 2 q2, qbar1 = 2 q1,
    qbar2 = 4 q2 (2 cos 2x = 4 cos^2 x - 2), where q0 = sum A_k^2,
    q1 = A0 A1 + A1 A2, q2 = A0 A2 (eqn:symbol_h_gen_poly)."""
    A0, A1, A2 = [np.asarray(B.todense()) if sp.issparse(B) else B for B in blocks]
    q0 = A0 @ A0 + A1 @ A1 + A2 @ A2
    q1 = A0 @ A1 + A1 @ A2
    q2 = A0 @ A2
    Pn = tridiag_half(n)
    In = np.eye(n)
    M2 = np.kron(In, q0 - 2 * q2) + np.kron(Pn, 2 * q1) + np.kron(Pn @ Pn, 4 * q2)
    return sqrtm_spd(M2)


def qbar_general(blocks):
    """qbar_0..qbar_l of def:matrix_P_gen for any l: eqn:symbol_h_gen_poly gives
    |ghat|^2 = q_0 + sum_{j >= 1} q_j 2 cos(j x) with q_j = sum_k A_(k) A_(k+j) (the blocks
    are symmetric and commute), and 2 cos(j x) = 2 T_j(cos x) (Chebyshev polynomials), so
    qbar_k collects the coefficient of cos^k x."""
    from numpy.polynomial import chebyshev as C
    A = [np.asarray(B.todense()) if sp.issparse(B) else np.asarray(B) for B in blocks]
    l = len(A) - 1
    q = [sum(A[k] @ A[k + j] for k in range(l + 1 - j)) for j in range(l + 1)]
    qbar = [np.zeros_like(A[0]) for _ in range(l + 1)]
    qbar[0] = qbar[0] + q[0]
    for j in range(1, l + 1):
        cj = C.cheb2poly([0.0] * j + [1.0])        # T_j in powers of cos x
        for k, c in enumerate(cj):
            if c != 0.0:
                qbar[k] = qbar[k] + 2.0 * c * q[j]
    return qbar


def Phat_dense_general(blocks, n: int) -> np.ndarray:
    """Phat = sqrt(sum_k P_n^k (x) qbar_k) of def:matrix_P_gen for any l."""
    qb = qbar_general(blocks)
    Pn = tridiag_half(n)
    M2 = np.zeros((n * qb[0].shape[0],) * 2)
    Pk = np.eye(n)
    for k in range(len(qb)):
        M2 = M2 + np.kron(Pk, qb[k])
        Pk = Pk @ Pn
    return sqrtm_spd(M2)


# ---------------------------------------------------------------- P_theta

def ptheta_eigs(n: int, theta: float):
    """(eta_j, zeta_j): eigenvalues of H and H_theta in S_n's order."""
    ph = phi(n)
    eta = 2.0 * np.sin(ph / 2.0)
    zeta = np.sqrt(theta ** 2 + (1 - theta) ** 2 + 2 * theta * (1 - theta) * np.cos(ph))
    return eta, zeta


def sigma_ptheta(mu: np.ndarray, n: int, tau: float, theta: float) -> np.ndarray:
    """Eigenvalues eta_j + tau zeta_j mu_k of P_theta when K = U diag(mu) U^T (constant a):
    then every per-mode block of Sec. 3.1.4 is diagonal in the spatial sine basis and
    P_theta^{-1} takes the same three steps as P_H with these values.  Shape (n, len(mu))."""
    eta, zeta = ptheta_eigs(n, theta)
    return eta[:, None] + tau * zeta[:, None] * np.asarray(mu, dtype=np.float64)[None, :]


def ptheta_dense(K, n: int, tau: float, theta: float) -> np.ndarray:
    """P_theta = H (x) I + H_theta (x) tau K assembled with dense matrix square roots."""
    T2 = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    Tt = ((theta ** 2 + (1 - theta) ** 2) * np.eye(n)
          + theta * (1 - theta) * (np.eye(n, k=1) + np.eye(n, k=-1)))
    H = sqrtm_spd(T2)
    Ht = sqrtm_spd(Tt)
    Kd = np.asarray(K.todense()) if sp.issparse(K) else K
    return np.kron(H, np.eye(Kd.shape[0])) + np.kron(Ht, tau * Kd)


def pinv_ptheta_exact(v: np.ndarray, K, n: int, tau: float, theta: float) -> np.ndarray:
    """Three steps of Sec. 3.1.4: time DST, per-mode solve (eta_j I + tau zeta_j K), time DST."""
    m = K.shape[0]
    eta, zeta = ptheta_eigs(n, theta)
    vt = dst(np.asarray(v, dtype=np.float64).reshape(n, m), axis=0)
    zt = np.empty_like(vt)
    I = sp.identity(m, format="csc")
    for j in range(n):
        zt[j] = spla.spsolve((eta[j] * I + tau * zeta[j] * K).tocsc(), vt[j])
    return dst(zt, axis=0).reshape(-1)


def chebyshev(apply_A, apply_Binv, r: np.ndarray, k: int, lo: float, hi: float) -> np.ndarray:
    """k steps of Chebyshev acceleration from x = 0 for A x = r with preconditioner B,
    given bounds lo <= eig(B^{-1} A) <= hi.  Uses k applications of B^{-1} and k - 1
    of A, so the result is p(B^{-1} A) B^{-1} r for one fixed polynomial p of degree
    k - 1 (positive on [lo, hi]): a fixed SPD operator, as MINRES requires of its
    preconditioner.  When lo == hi, B^{-1} A = lo I and the result is B^{-1} r / lo."""
    c = 0.5 * (hi + lo)
    d = 0.5 * (hi - lo)
    if d == 0.0:
        return apply_Binv(r) / c
    s1 = c / d
    rho = 1.0 / s1
    res = r.copy()
    dvec = apply_Binv(res) / c
    x = np.zeros_like(r)
    for i in range(k):
        x = x + dvec
        if i == k - 1:
            break
        res = res - apply_A(dvec)
        rho_new = 1.0 / (2.0 * s1 - rho)
        dvec = rho_new * rho * dvec + (2.0 * rho_new / d) * apply_Binv(res)
        rho = rho_new
    return x


def cheb_params(a_min: float, a_max: float):
    """abar and the bounds [lo, hi] on eig(B_j^{-1} A_j) for every mode j.

    With a_min <= a <= a_max on all faces, a_min K_lap <= K(a) <= a_max K_lap, so the
    Rayleigh quotient of (eta I + tau zeta K(a), eta I + tau zeta abar K_lap) lies in
    [min(1, a_min/abar), max(1, a_max/abar)].  abar is the midpoint of [a_min, a_max]."""
    abar = 0.5 * (a_min + a_max)
    return abar, min(1.0, a_min / abar), max(1.0, a_max / abar)


def pinv_ptheta_cheb(v: np.ndarray, K, N: int, dim: int, n: int, tau: float, theta: float,
                     k: int, a_min: float, a_max: float) -> np.ndarray:
    """P_theta^{-1} v with each per-mode solve replaced by k Chebyshev steps whose
    inner preconditioner eta_j I + tau zeta_j abar K_lap is applied by the spatial
    sine transforms (1D, 2D or 3D)."""
    from .spatial import mu_const
    m = K.shape[0]
    eta, zeta = ptheta_eigs(n, theta)
    abar, lo, hi = cheb_params(a_min, a_max)
    mu = mu_const(N, dim)
    sp_axes = tuple(range(dim))
    shp = (N,) * dim
    vt = dst(np.asarray(v, dtype=np.float64).reshape(n, m), axis=0)
    zt = np.empty_like(vt)
    for j in range(n):
        diag = eta[j] + tau * zeta[j] * abar * mu

        def binv(r, diag=diag):
            rt = dstn(r.reshape(shp), sp_axes)
            return dstn(rt / diag.reshape(shp), sp_axes).reshape(-1)

        def amul(x, j=j):
            return eta[j] * x + tau * zeta[j] * (K @ x)

        zt[j] = chebyshev(amul, binv, vt[j], k, lo, hi)
    return dst(zt, axis=0).reshape(-1)
