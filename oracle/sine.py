"""Sine transforms (oracle; test infrastructure only).

S_n = sqrt(2/(n+1)) [sin(i j pi/(n+1))]_{i,j=1..n} is the symmetric, orthogonal
discrete sine transform matrix of Sec. 3.1.1 (eqn:matrix_tri_p); it diagonalises
P_n = tridiag(1/2, 0, 1/2) with eigenvalues cos(j pi/(n+1)).
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def dst_matrix(n: int) -> np.ndarray:
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))


def tridiag_half(n: int) -> np.ndarray:
    """P_n of eqn:matrix_tri_p."""
    P = np.zeros((n, n))
    i = np.arange(n - 1)
    P[i, i + 1] = 0.5
    P[i + 1, i] = 0.5
    return P


def cos_phi(n: int) -> np.ndarray:
    """Eigenvalues cos(phi_j), phi_j = j pi/(n+1), j = 1..n, of P_n in S_n's order."""
    return np.cos(np.arange(1, n + 1, dtype=np.float64) * np.pi / (n + 1))


def dst(x: np.ndarray, axis: int = -1, workers: int = 1) -> np.ndarray:
    """Orthonormal DST-I along one axis (equal to multiplying by S_n)."""
    return scipy.fft.dst(x, type=1, norm="ortho", axis=axis, workers=workers)


def dstn(x: np.ndarray, axes, workers: int = 1) -> np.ndarray:
    return scipy.fft.dstn(x, type=1, norm="ortho", axes=axes, workers=workers)
