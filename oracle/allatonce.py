"""All-at-once systems (oracle; test infrastructure only).

theta-method (Sec. 1, eq. theta): T_H is block lower-bidiagonal Toeplitz with
A0 = M + theta tau K on the diagonal and A1 = -M + (1-theta) tau K below it
(eqn:symbol_h); f_H's first block carries (M - (1-theta) tau K) u0.
BDF2 (Sec. 4, eqn:matrix_gen with l = 2): A0 = 1.5 I + tau K, A1 = -2 I,
A2 = 0.5 I (the standard two-step backward difference multiplied by tau; the
paper leaves the blocks unnamed), right-hand side given directly; BDF-l (l = 3, 4)
the same from the l-step backward difference formula (bdf_coefficients).
Y = Y_n (x) I_m is the time flip of eqn:main_system; Y T is symmetric.
M = I throughout (finite differences, Sec. 5).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def theta_blocks(K, tau: float, theta: float):
    I = sp.identity(K.shape[0], format="csr")
    return [(I + theta * tau * K).tocsr(), (-I + (1.0 - theta) * tau * K).tocsr()]


def bdf2_blocks(K, tau: float):
    I = sp.identity(K.shape[0], format="csr")
    return [(1.5 * I + tau * K).tocsr(), (-2.0 * I).tocsr(), (0.5 * I).tocsr()]


def bdf_coefficients(l: int) -> np.ndarray:
    """alpha_0..alpha_l of the l-step backward difference formula (Sec. 4 leaves the blocks
    A_(k) to the scheme): tau u'(t_k) is approximated by sum_j nabla^j u^k / j over
    j = 1..l, nabla u^k = u^k - u^{k-1}; expanding nabla^j = sum_k binom(j, k) (-1)^k E^k
    (E u^k = u^{k-1}) gives alpha_k = (-1)^k sum_{j >= max(k, 1)} binom(j, k) / j."""
    from math import comb
    a = np.zeros(l + 1)
    for j in range(1, l + 1):
        for k in range(j + 1):
            a[k] += (-1) ** k * comb(j, k) / j
    return a


def bdf_blocks(K, tau: float, l: int):
    """Blocks of eqn:matrix_gen for BDF-l with M = I, multiplied by tau:
    A_(0) = alpha_0 I + tau K, A_(k) = alpha_k I (k = 1..l); start-up values enter the
    right-hand side, so the matrix stays block Toeplitz."""
    a = bdf_coefficients(l)
    I = sp.identity(K.shape[0], format="csr")
    return [(a[0] * I + tau * K).tocsr()] + [(a[k] * I).tocsr() for k in range(1, l + 1)]


def assemble_T(blocks, n: int) -> sp.csr_matrix:
    """Block lower-banded Toeplitz matrix sum_l (E_n^l (x) A_l), E_n = ones on the
    first subdiagonal (eq. theta and eqn:matrix_gen)."""
    T = None
    for l, A in enumerate(blocks):
        if l >= n:
            break
        E = sp.diags([np.ones(n - l)], [-l], shape=(n, n), format="csr")
        term = sp.kron(E, A, format="csr")
        T = term if T is None else T + term
    return T.tocsr()


def flip(n: int, m: int) -> sp.csr_matrix:
    """Y = Y_n (x) I_m, Y_n the anti-identity (eqn:main_system)."""
    Yn = sp.csr_matrix(np.fliplr(np.eye(n)))
    return sp.kron(Yn, sp.identity(m), format="csr")


def flip_vec(x: np.ndarray, n: int) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x).reshape(n, -1)[::-1].reshape(-1))


def rhs_theta(f: np.ndarray, u0: np.ndarray, K, tau: float, theta: float) -> np.ndarray:
    """f_H of Sec. 1: block k (k = 1..n) is theta tau f^(k) + (1-theta) tau f^(k-1);
    block 1 adds (M - (1-theta) tau K) u0.  f has shape (n+1, m)."""
    f = np.asarray(f, dtype=np.float64)
    b = theta * tau * f[1:] + (1.0 - theta) * tau * f[:-1]
    b = b.copy()
    b[0] += u0 - (1.0 - theta) * tau * (K @ u0)
    return b.reshape(-1)


def apply_T(blocks, x: np.ndarray, n: int) -> np.ndarray:
    """(T x)_k = sum_l A_l x_{k-l} without assembling T."""
    X = np.asarray(x).reshape(n, -1)
    out = np.zeros_like(X)
    for l, A in enumerate(blocks):
        if l >= n:
            break
        out[l:] += (A @ X[: n - l].T).T
    return out.reshape(-1)


def apply_YT(blocks, x: np.ndarray, n: int) -> np.ndarray:
    return flip_vec(apply_T(blocks, x, n), n)


def sequential(blocks, b: np.ndarray, n: int) -> np.ndarray:
    """Exact u = T^{-1} b by forward block substitution, one sparse SPD solve per
    time level (the sequential stepping of Sec. 1)."""
    B = np.asarray(b).reshape(n, -1)
    lu = spla.splu(blocks[0].tocsc())
    U = np.zeros_like(B)
    for k in range(n):
        r = B[k].copy()
        for l in range(1, len(blocks)):
            if k - l >= 0:
                r -= blocks[l] @ U[k - l]
        U[k] = lu.solve(r)
    return U.reshape(-1)


def sequential_theta_steps(f, u0, K, tau, theta):
    """Plain theta-method time stepping of Sec. 1:
    (M + theta tau K) u^{k+1} = (M - (1-theta) tau K) u^k + theta tau f^{k+1} + (1-theta) tau f^k."""
    m = K.shape[0]
    I = sp.identity(m, format="csc")
    lu = spla.splu((I + theta * tau * K).tocsc())
    Bm = (I - (1.0 - theta) * tau * K).tocsr()
    u = np.asarray(u0, dtype=np.float64).copy()
    out = []
    for k in range(f.shape[0] - 1):
        u = lu.solve(Bm @ u + theta * tau * f[k + 1] + (1.0 - theta) * tau * f[k])
        out.append(u)
    return np.concatenate(out)
