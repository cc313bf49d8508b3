"""Oracle pins for the 3D problems of Sec. 5 (Example 3: 7-point stencil, 3D spatial sine
transform, so a 4D transform with time).

  * the 3D stiffness matrix against node-by-node flux sums (variable faces) and against
    the Kronecker sum of three 1D Laplacians (constant a);
  * S_N (x) S_N (x) S_N diagonalises it with the closed-form eigenvalues;
  * the averaged Kbar keeps the literal means of K's diagonals and is sine-diagonal;
  * P_H^{-1} of the three-step form equals the dense square root of def:matrix_P;
  * for constant a, P_theta is diagonal in the 4D sine basis (eta_j + tau zeta_j mu_k) and
    equals the exact per-mode solves of Sec. 3.1.4 and the dense H (x) I + H_theta (x) tau K;
  * MINRES iteration counts against the printed P_H and P_theta columns of Tables 6 and 7:
    small rows live, every row through golden/paper_oracle_counts_3d.txt (written by a
    script that calls only the oracle).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import precond as pc
from oracle import sine, spatial
from oracle.system import System

HERE = os.path.dirname(os.path.abspath(__file__))


def _faces3(N, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.5, 2.0, (N, N, N + 1)), rng.uniform(0.5, 2.0, (N, N + 1, N)),
            rng.uniform(0.5, 2.0, (N + 1, N, N)))


@pytest.mark.parametrize("N", [1, 2, 4])
def test_stiffness_3d_equals_flux_sums(N):
    """(K u)_p = sum over the six faces of node p of a_face (u_p - u_neighbour) / h^2, with
    u = 0 beyond the boundary, evaluated node by node."""
    ax, ay, az = _faces3(N, 3 + N)
    K = spatial.stiffness(N, 3, ax, ay, az)
    u = np.random.default_rng(5).standard_normal((N, N, N))
    h2 = (1.0 / (N + 1)) ** 2

    def val(k, j, i):
        return u[k, j, i] if 0 <= i < N and 0 <= j < N and 0 <= k < N else 0.0

    ref = np.zeros((N, N, N))
    for k in range(N):
        for j in range(N):
            for i in range(N):
                s = ax[k, j, i] * (u[k, j, i] - val(k, j, i - 1)) + ax[k, j, i + 1] * (u[k, j, i] - val(k, j, i + 1))
                s += ay[k, j, i] * (u[k, j, i] - val(k, j - 1, i)) + ay[k, j + 1, i] * (u[k, j, i] - val(k, j + 1, i))
                s += az[k, j, i] * (u[k, j, i] - val(k - 1, j, i)) + az[k + 1, j, i] * (u[k, j, i] - val(k + 1, j, i))
                ref[k, j, i] = s / h2
    assert np.abs(K @ u.reshape(-1) - ref.reshape(-1)).max() <= 1e-12 * np.abs(ref).max()
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() == 0.0


def test_stiffness_3d_constant_is_kronecker_sum():
    N, a = 5, 0.3
    h2inv = (N + 1) ** 2
    K1 = a * h2inv * sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.identity(N)
    ref = sp.kron(sp.kron(I, I), K1) + sp.kron(sp.kron(I, K1), I) + sp.kron(sp.kron(K1, I), I)
    faces = spatial.const_faces(N, 3, a)
    K = spatial.stiffness(N, 3, *faces)
    assert np.abs((K - ref).toarray()).max() <= 1e-12 * a * h2inv


def test_sine_transform_diagonalises_3d():
    N = 4
    K = spatial.stiffness(N, 3).toarray()
    S = sine.dst_matrix(N)
    U = np.kron(np.kron(S, S), S)
    mu = spatial.mu_const(N, 3)
    assert np.abs(U @ K @ U - np.diag(mu)).max() < 1e-10 * mu.max()
    assert np.abs(np.sort(mu) - np.linalg.eigvalsh(K)).max() < 1e-10 * mu.max()
    # the oracle's 3D transform is that Kronecker product
    x = np.random.default_rng(6).standard_normal(N ** 3)
    assert np.abs(sine.dstn(x.reshape(N, N, N), (0, 1, 2)).reshape(-1) - U @ x).max() < 1e-13


def test_kbar_3d_literal_means():
    N = 4
    ax, ay, az = _faces3(N, 7)
    K = spatial.stiffness(N, 3, ax, ay, az).toarray()
    h2 = (1.0 / (N + 1)) ** 2
    d, cx, cy, cz = spatial.kbar_params3(N, ax, ay, az)
    at = lambda k, j, i: (k * N + j) * N + i
    assert abs(d - np.mean(np.diag(K)) * h2) < 1e-12
    xc = [K[at(k, j, i), at(k, j, i + 1)] for k in range(N) for j in range(N) for i in range(N - 1)]
    yc = [K[at(k, j, i), at(k, j + 1, i)] for k in range(N) for j in range(N - 1) for i in range(N)]
    zc = [K[at(k, j, i), at(k + 1, j, i)] for k in range(N - 1) for j in range(N) for i in range(N)]
    assert abs(cx + np.mean(xc) * h2) < 1e-12
    assert abs(cy + np.mean(yc) * h2) < 1e-12
    assert abs(cz + np.mean(zc) * h2) < 1e-12
    S = sine.dst_matrix(N)
    U = np.kron(np.kron(S, S), S)
    Kb = spatial.kbar_matrix(N, 3, ax, ay, az).toarray()
    mu = spatial.mu_kbar(N, 3, ax, ay, az)
    assert np.abs(U @ Kb @ U - np.diag(mu)).max() < 1e-10 * np.abs(mu).max()
    # constant faces: Kbar = K and its eigenvalues are the closed form
    f = spatial.const_faces(N, 3, 0.7)
    assert np.abs(spatial.kbar_matrix(N, 3, *f).toarray() - spatial.stiffness(N, 3, *f).toarray()).max() < 1e-9
    assert np.abs(spatial.mu_kbar(N, 3, *f) - spatial.mu_const(N, 3, 0.7)).max() < 1e-9 * 0.7 * (N + 1) ** 2


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_PH_3d_three_step_equals_dense(theta):
    """def:matrix_P: P_H = sqrt(T_n[|g|^2]) with the blocks of the 3D theta scheme, assembled
    densely; its inverse against the transform-divide-transform form."""
    N, n = 3, 4
    s = System(3, N, n, theta=theta)
    A0, A1 = [np.asarray(B.todense()) if sp.issparse(B) else B for B in s.blocks]
    P = pc.PH_dense(A0, A1, n)
    v = np.random.default_rng(8).standard_normal(n * s.m)
    ref = np.linalg.solve(P, v)
    assert np.abs(s.apply_Pinv(v) - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.7])
def test_Ptheta_3d_constant_is_sine_diagonal(theta):
    """Constant a: the per-mode blocks eta_j I + tau zeta_j K share K's eigenvectors, so
    P_theta^{-1} divides by eta_j + tau zeta_j mu_k in the 4D sine basis; this equals the
    exact per-mode solves, the Chebyshev form (its inner preconditioner is exact here) and
    the dense definition."""
    N, n, a = 3, 5, 0.4
    faces = spatial.const_faces(N, 3, a)
    s = System(3, N, n, theta=theta, ax=faces[0], ay=faces[1], az=faces[2], precond="PTHETA_CHEB", cheb_k=3)
    v = np.random.default_rng(9).standard_normal(n * s.m)
    sig = pc.sigma_ptheta(spatial.mu_const(N, 3, a), n, s.tau, theta)
    z = pc.pinv_spectral(v, sig, n, N, 3)
    exact = pc.pinv_ptheta_exact(v, s.K, n, s.tau, theta)
    dense = np.linalg.solve(pc.ptheta_dense(s.K, n, s.tau, theta), v)
    assert np.abs(z - dense).max() < 1e-11 * np.abs(dense).max()
    assert np.abs(exact - dense).max() < 1e-11 * np.abs(dense).max()
    assert np.abs(s.apply_Pinv(v) - dense).max() < 1e-11 * np.abs(dense).max()


def test_example3_rhs_and_direct_solution():
    """f_H of the theta scheme in 3D carries (I - (1 - theta) tau K) u0 on block 1; with f = 0
    each 3D sine mode of the direct solution follows the scalar theta recurrence, i.e. is
    multiplied per step by the amplification factor (1 - (1 - theta) tau mu) / (1 + theta tau mu)."""
    N, n = 7, 16
    p = W.example3(N, n, 0.5)
    s = System(3, N, n, theta=0.5, ax=p.ax, ay=p.ay, az=p.az)
    b = s.rhs(p.f, p.u0)
    ref0 = p.u0 - 0.5 * s.tau * (s.K @ p.u0)
    assert np.abs(b[:s.m] - ref0).max() < 1e-15 and np.abs(b[s.m:]).max() == 0.0
    u = s.solve_direct(b).reshape(n, s.m)
    mu = spatial.mu_const(N, 3, 1e-3)
    g = (1 - 0.5 * s.tau * mu) / (1 + 0.5 * s.tau * mu)
    c0 = sine.dstn(p.u0.reshape(N, N, N), (0, 1, 2)).reshape(-1)
    for k in (0, 5, n - 1):
        ck = sine.dstn(u[k].reshape(N, N, N), (0, 1, 2)).reshape(-1)
        assert np.abs(ck - g ** (k + 1) * c0).max() < 1e-14


def _rows():
    with open(os.path.join(HERE, "golden", "paper_tables_3d.txt")) as fh:
        return [l.split() for l in fh if l.strip() and not l.startswith("#")]


@pytest.mark.parametrize("row", [r for r in _rows() if int(r[4]) <= 60000], ids=lambda r: f"{r[0]}-n{r[2]}-m{r[3]}")
def test_example3_small_rows_match_printed(row):
    tab, theta, n, mp1 = row[0], float(row[1]), int(row[2]), int(row[3])
    N = mp1 - 1
    assert n * N ** 3 == int(row[4])
    p = W.example3(N, n, theta)
    its = []
    for pre in ("PH", "PTHETA_CHEB"):
        s = System(3, N, n, theta=theta, ax=p.ax, ay=p.ay, az=p.az, precond=pre)
        r = s.solve(s.rhs(p.f, p.u0), rtol=1e-6, maxit=200)
        assert r.status == "converged"
        its.append(r.iters)
    assert its[0] == int(row[6]), (row, its)
    # P_theta: the printed count, or one more than the oracle's on the Crank-Nicolson rows
    # listed in the golden counts (the paper's per-mode solver is not specified)
    assert its[1] in (int(row[8]), int(row[8]) - 1), (row, its)


def test_example3_golden_counts_against_printed():
    """Every row of Tables 6 and 7: the oracle's P_H count equals the printed one (32 of 32);
    its P_theta count equals the printed one on all 16 backward Euler rows and on 11 of the 16
    Crank-Nicolson rows, and is 1 or 2 lower on the other five (the paper does not say how its
    per-mode systems are solved; here they are solved exactly)."""
    path = os.path.join(HERE, "golden", "paper_oracle_counts_3d.txt")
    if not os.path.exists(path):
        pytest.skip("golden/paper_oracle_counts_3d.txt not written yet")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 32
    printed = {(r[0], int(r[2]), int(r[3])): (int(r[6]), int(r[8])) for r in _rows()}
    off = []
    for r in rows:
        key = (r[0], int(r[1]), int(r[2]))
        assert printed[key] == (int(r[5]), int(r[6]))
        assert int(r[3]) == int(r[5]), r
        if int(r[4]) != int(r[6]):
            assert r[0] == "T7" and int(r[6]) - 2 <= int(r[4]) < int(r[6]), r
            off.append(key)
    assert len(off) == 5, off
