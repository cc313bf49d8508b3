"""Finite-difference spatial operators (oracle; test infrastructure only).

K(a) is the matrix of eqn:matrix_Km_va (Sec. 3.1.1): in 1D the tridiagonal
matrix with diagonal (a_{i-1/2} + a_{i+1/2})/h^2 and off-diagonals -a_{i+1/2}/h^2;
in 2D the same construction applied along x (rows) and along y (columns) and
summed (the 5-point stencil).  M = I for finite differences (Sec. 5).

In 3D (Example 3 of Sec. 5) the same construction along z gives the 7-point stencil.

Face arrays follow the grid convention of the ``workloads`` module:
1D ax[i] ~ a((i+1/2)h), i = 0..N;  2D ax[j, i] ~ a((i+1/2)h, (j+1)h) (N x (N+1)),
ay[j, i] ~ a((i+1)h, (j+1/2)h) ((N+1) x N);  3D ax[k, j, i] ~ a((i+1/2)h, (j+1)h, (k+1)h)
(N x N x (N+1)), ay[k, j, i] (N x (N+1) x N), az[k, j, i] ~ a((i+1)h, (j+1)h, (k+1/2)h)
((N+1) x N x N).  Unknowns are ordered x fastest, z slowest.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def const_faces(N: int, dim: int, a: float = 1.0):
    """(ax, ay) in 1D/2D (ay None in 1D), (ax, ay, az) in 3D, all equal to a."""
    if dim == 1:
        return np.full(N + 1, a), None
    if dim == 2:
        return np.full((N, N + 1), a), np.full((N + 1, N), a)
    return np.full((N, N, N + 1), a), np.full((N, N + 1, N), a), np.full((N + 1, N, N), a)


def faces_from_nodal(a_nodal: np.ndarray, dim: int):
    """Face value = mean of the two nodal values it joins (nodal grid includes the
    boundary).  The paper only prints face values a_{j+1/2}; taking the mean of
    the endpoint nodes is the reading used for a nodally given coefficient."""
    a = np.asarray(a_nodal, dtype=np.float64)
    if dim == 1:
        return 0.5 * (a[:-1] + a[1:]), None
    ax = 0.5 * (a[1:-1, :-1] + a[1:-1, 1:])     # between (J, I) and (J, I+1), J = 1..N
    ay = 0.5 * (a[:-1, 1:-1] + a[1:, 1:-1])     # between (J, I) and (J+1, I), I = 1..N
    return np.ascontiguousarray(ax), np.ascontiguousarray(ay)


def stiffness(N: int, dim: int, ax=None, ay=None, az=None) -> sp.csr_matrix:
    """K(a) of eqn:matrix_Km_va; a == 1 when the face arrays are None."""
    h2 = (1.0 / (N + 1)) ** 2
    if dim == 3:
        return _stiffness3(N, ax, ay, az)
    if ax is None:
        ax, ay = const_faces(N, dim)
    if dim == 1:
        ax = np.asarray(ax, dtype=np.float64)
        main = (ax[:-1] + ax[1:]) / h2
        off = -ax[1:-1] / h2
        return sp.diags([off, main, off], [-1, 0, 1], shape=(N, N), format="csr")
    ax = np.asarray(ax, dtype=np.float64)
    ay = np.asarray(ay, dtype=np.float64)
    idx = np.arange(N * N).reshape(N, N)
    diag = (ax[:, :-1] + ax[:, 1:] + ay[:-1, :] + ay[1:, :]) / h2
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    # x couplings between (j, i) and (j, i+1) across face ax[j, i+1]
    cx = -ax[:, 1:-1] / h2
    rows += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    cols += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    vals += [cx.ravel(), cx.ravel()]
    # y couplings between (j, i) and (j+1, i) across face ay[j+1, i]
    cy = -ay[1:-1, :] / h2
    rows += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals += [cy.ravel(), cy.ravel()]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N * N, N * N))
    return K.tocsr()


def _stiffness3(N: int, ax=None, ay=None, az=None) -> sp.csr_matrix:
    """3D: every interior node couples to its six neighbours across the faces between
    them; the diagonal is the sum of its six face values (all over h^2)."""
    h2 = (1.0 / (N + 1)) ** 2
    if ax is None:
        ax, ay, az = const_faces(N, 3)
    ax, ay, az = (np.asarray(a, dtype=np.float64) for a in (ax, ay, az))
    idx = np.arange(N ** 3).reshape(N, N, N)          # [k, j, i], i = x fastest
    diag = (ax[:, :, :-1] + ax[:, :, 1:] + ay[:, :-1, :] + ay[:, 1:, :] + az[:-1] + az[1:]) / h2
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [diag.ravel()]
    for lo, hi, c in ((idx[:, :, :-1], idx[:, :, 1:], -ax[:, :, 1:-1] / h2),
                      (idx[:, :-1, :], idx[:, 1:, :], -ay[:, 1:-1, :] / h2),
                      (idx[:-1], idx[1:], -az[1:-1] / h2)):
        rows += [lo.ravel(), hi.ravel()]
        cols += [hi.ravel(), lo.ravel()]
        vals += [c.ravel(), c.ravel()]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N ** 3, N ** 3))
    return K.tocsr()


def face_difference(N: int, dim: int):
    """Difference operators across faces: (D u)_e = u(right/upper node) - u(left/lower
    node), with the Dirichlet boundary value 0.  Returns (Dx, Dy) as sparse matrices
    mapping interior unknowns to x-faces and y-faces (same ordering as ax, ay)."""
    e = np.ones(N + 1)
    # row i (face i+1/2, i = 0..N) = u[i] - u[i-1] in 0-based interior indices
    D1 = sp.diags([e[:N], -e[:N]], [0, -1], shape=(N + 1, N), format="csr")
    if dim == 1:
        return D1, None
    I = sp.identity(N, format="csr")
    Dx = sp.kron(I, D1, format="csr")      # faces ordered (j, i) with i fastest -> (N, N+1)
    Dy = sp.kron(D1, I, format="csr")      # faces ordered (j, i) -> (N+1, N)
    return Dx, Dy


def laplacian_eigs_1d(N: int) -> np.ndarray:
    """Eigenvalues (4/h^2) sin^2(k pi / (2(N+1))), k = 1..N, of tridiag(-1, 2, -1)/h^2,
    whose eigenvectors are the columns of the sine matrix S_N."""
    k = np.arange(1, N + 1, dtype=np.float64)
    return 4.0 * (N + 1) ** 2 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2


def mu_const(N: int, dim: int, a: float = 1.0) -> np.ndarray:
    """Eigenvalues of K for constant a in the sine basis, flattened x fastest."""
    l1 = laplacian_eigs_1d(N)
    if dim == 1:
        return a * l1
    if dim == 2:
        return a * (l1[None, :] + l1[:, None]).reshape(-1)
    return a * (l1[None, None, :] + l1[None, :, None] + l1[:, None, None]).reshape(-1)


def kbar_params(N: int, dim: int, ax, ay=None):
    """Averaged-Toeplitz reading of Sec. 3.1.1: average K's entries along each of its
    diagonals.  Returns (d, cx, cy) in units of 1/h^2: d = mean of h^2 diag(K),
    cx (cy) = mean of the coupling coefficients along x (y), i.e. of the interior
    faces; the structural zeros of the 2D band are not averaged in, so that the
    result keeps the Kronecker-sum form that the 2D sine transform diagonalises."""
    ax = np.asarray(ax, dtype=np.float64)
    if dim == 1:
        d = float(np.mean(ax[:-1] + ax[1:]))
        cx = float(np.mean(ax[1:-1])) if N > 1 else 0.0
        return d, cx, 0.0
    ay = np.asarray(ay, dtype=np.float64)
    d = float(np.mean(ax[:, :-1] + ax[:, 1:] + ay[:-1, :] + ay[1:, :]))
    cx = float(np.mean(ax[:, 1:-1])) if N > 1 else 0.0
    cy = float(np.mean(ay[1:-1, :])) if N > 1 else 0.0
    return d, cx, cy


def kbar_params3(N: int, ax, ay, az):
    """3D form of kbar_params: (d, cx, cy, cz), the mean of h^2 diag(K) and the means of
    the interior x-, y- and z-face coefficients."""
    ax, ay, az = (np.asarray(a, dtype=np.float64) for a in (ax, ay, az))
    d = float(np.mean(ax[:, :, :-1] + ax[:, :, 1:] + ay[:, :-1, :] + ay[:, 1:, :] + az[:-1] + az[1:]))
    if N == 1:
        return d, 0.0, 0.0, 0.0
    return d, float(np.mean(ax[:, :, 1:-1])), float(np.mean(ay[:, 1:-1, :])), float(np.mean(az[1:-1]))


def kbar_matrix(N: int, dim: int, ax, ay=None, az=None) -> sp.csr_matrix:
    h2 = (1.0 / (N + 1)) ** 2
    E = sp.diags([np.ones(N - 1), np.ones(N - 1)], [-1, 1], shape=(N, N), format="csr")
    I = sp.identity(N, format="csr")
    if dim == 3:
        d, cx, cy, cz = kbar_params3(N, ax, ay, az)
        return ((d * sp.identity(N ** 3) - cx * sp.kron(sp.kron(I, I), E) - cy * sp.kron(sp.kron(I, E), I)
                 - cz * sp.kron(sp.kron(E, I), I)) / h2).tocsr()
    d, cx, cy = kbar_params(N, dim, ax, ay)
    if dim == 1:
        return ((d * I - cx * E) / h2).tocsr()
    return ((d * sp.identity(N * N) - cx * sp.kron(I, E) - cy * sp.kron(E, I)) / h2).tocsr()


def mu_kbar(N: int, dim: int, ax, ay=None, az=None) -> np.ndarray:
    """Eigenvalues of Kbar in the sine basis, flattened x fastest.

    d - 2 c cos(t) is written (d - 2 c) + 4 c sin^2(t/2) to avoid cancellation for
    the smooth modes; for constant a it equals the closed form of mu_const."""
    s2 = np.sin(np.arange(1, N + 1, dtype=np.float64) * np.pi / (2.0 * (N + 1))) ** 2
    h2inv = float(N + 1) ** 2
    if dim == 3:
        d, cx, cy, cz = kbar_params3(N, ax, ay, az)
        return (((d - 2.0 * (cx + cy + cz)) + 4.0 * cx * s2[None, None, :] + 4.0 * cy * s2[None, :, None]
                 + 4.0 * cz * s2[:, None, None]) * h2inv).reshape(-1)
    d, cx, cy = kbar_params(N, dim, ax, ay)
    if dim == 1:
        return ((d - 2.0 * cx) + 4.0 * cx * s2) * h2inv
    return (((d - 2.0 * cx - 2.0 * cy) + 4.0 * cx * s2[None, :] + 4.0 * cy * s2[:, None]) * h2inv).reshape(-1)


def coef_bounds(N: int, dim: int, ax, ay=None, az=None):
    """(a_min, a_max) over all face coefficients."""
    if ax is None:
        return 1.0, 1.0
    vals = [np.asarray(ax).ravel()]
    if dim >= 2:
        vals.append(np.asarray(ay).ravel())
    if dim == 3:
        vals.append(np.asarray(az).ravel())
    v = np.concatenate(vals)
    return float(v.min()), float(v.max())
