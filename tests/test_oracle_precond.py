"""Pins of the preconditioners against dense matrix functions and the paper's
algebraic statements (Sec. 3-4).  All dense checks run on tiny grids."""
import numpy as np
import pytest

from oracle import allatonce as aao
from oracle import precond as pc
from oracle import sine, spatial
from oracle.system import System


def _rand_faces(N, dim, seed=0, lo=0.5, hi=2.0):
    rng = np.random.default_rng(seed)
    if dim == 1:
        return rng.uniform(lo, hi, N + 1), None
    return rng.uniform(lo, hi, (N, N + 1)), rng.uniform(lo, hi, (N + 1, N))


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("dim,N,n", [(1, 5, 6), (2, 3, 5)])
def test_PH_dense_sqrtm_equals_dst_form(theta, dim, N, n):
    """def:matrix_P: sqrtm of the block tridiagonal T[|g|^2] equals the three-step form."""
    s = System(dim, N, n, theta=theta)
    A0, A1 = [B.toarray() for B in s.blocks]
    PH = pc.PH_dense(A0, A1, n)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(n * s.m)
    z = s.apply_Pinv(v)
    z_dense = np.linalg.solve(PH, v)
    assert np.abs(z - z_dense).max() <= 1e-12 * np.abs(z_dense).max()
    # eigenvalues of P_H are exactly sigma_{j,k}
    assert np.abs(np.sort(np.linalg.eigvalsh(PH)) - np.sort(s.sigma.ravel())).max() < 1e-12 * s.sigma.max()


def test_PH_square_structure():
    """P_H^2 = I (x) (A0^2 + A1^2) + P_n (x) 2 A0 A1 (Sec. 3.1.1)."""
    N, n = 4, 5
    s = System(1, N, n, theta=0.5)
    A0, A1 = [B.toarray() for B in s.blocks]
    PH = pc.PH_dense(A0, A1, n)
    rhs = np.kron(np.eye(n), A0 @ A0 + A1 @ A1) + np.kron(sine.tridiag_half(n), 2 * A0 @ A1)
    assert np.abs(PH @ PH - rhs).max() < 1e-11 * np.abs(rhs).max()


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_TtT_minus_PH2_is_last_block(theta):
    """lemma:rankC_P: T^T T - P_H^2 = diag(0, ..., 0, -A1^2)."""
    N, n = 3, 6
    ax, ay = _rand_faces(N, 2, 3)
    s = System(2, N, n, theta=theta, ax=ax, ay=ay)
    A0, A1 = [B.toarray() for B in s.blocks]
    T = s.assemble_T().toarray()
    D = T.T @ T - pc.block_tridiag_sq(A0, A1, n)
    m = s.m
    expect = np.zeros_like(D)
    expect[-m:, -m:] = -A1 @ A1
    assert np.abs(D - expect).max() < 1e-10 * np.abs(T).max() ** 2


@pytest.mark.parametrize("scheme", ["theta", "bdf2"])
def test_abs_preconditioner_eigs_pm1(scheme):
    """thm:absC / thm:absC_gen: sqrt(T^T T)^{-1} Y T is symmetric orthogonal, eigenvalues +-1."""
    N, n = 3, 5
    s = System(2, N, n, scheme=scheme, theta=0.5)
    T = s.assemble_T().toarray()
    Y = aao.flip(n, s.m).toarray()
    Q = np.linalg.solve(pc.sqrtm_spd(T.T @ T), Y @ T)
    assert np.abs(Q - Q.T).max() < 1e-10
    assert np.abs(Q @ Q.T - np.eye(len(Q))).max() < 1e-10
    ev = np.linalg.eigvals(Q)
    assert np.abs(np.abs(ev.real) - 1).max() < 1e-9 and np.abs(ev.imag).max() < 1e-9


def test_normal_equations_unit_eigenvalues():
    """thm:main_P_normal: (P_H^{-1} T)^T (P_H^{-1} T) = I + rank <= m, so at least
    m (n - 1) eigenvalues equal 1."""
    N, n = 5, 6
    s = System(1, N, n, theta=0.5)
    A0, A1 = [B.toarray() for B in s.blocks]
    PHi = np.linalg.inv(pc.PH_dense(A0, A1, n))
    T = s.assemble_T().toarray()
    M = (PHi @ T).T @ (PHi @ T)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert np.sum(np.abs(ev - 1) < 1e-8) >= s.m * (n - 1)


def test_eigen_cluster_outliers_flat_in_n():
    """thm:absP_main: eigenvalues of P_H^{-1} Y T cluster at +-1 with a number of
    outliers that does not grow with n (m fixed)."""
    N = 3
    counts = []
    for n in (8, 16, 32):
        s = System(1, N, n, theta=1.0, ax=np.full(N + 1, 0.05))
        A0, A1 = [B.toarray() for B in s.blocks]
        Y = aao.flip(n, s.m).toarray()
        ev = np.linalg.eigvals(np.linalg.solve(pc.PH_dense(A0, A1, n), Y @ s.assemble_T().toarray())).real
        counts.append(int(np.sum(np.minimum(np.abs(ev - 1), np.abs(ev + 1)) > 0.1)))
    assert max(counts) <= counts[0] + 1, counts


def test_bdf2_Phat_dense_equals_dst_form_and_corner_structure():
    """def:matrix_P_gen with qbar0 = q0 - 2 q2, qbar1 = 2 q1, qbar2 = 4 q2; its
    eigenvalues are |ghat(phi_j)|.  lemma:rankC_P_gen: That^T That - Phat^2 is
    supported in the first and last l m rows and columns."""
    N, n = 3, 7
    s = System(1, N, n, scheme="bdf2")
    Ph = pc.Phat_dense(s.blocks, n)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(n * s.m)
    assert np.abs(s.apply_Pinv(v) - np.linalg.solve(Ph, v)).max() < 1e-12 * np.abs(np.linalg.solve(Ph, v)).max()
    T = s.assemble_T().toarray()
    D = T.T @ T - Ph @ Ph
    m, l = s.m, 2
    inner = D[l * m:(n - l) * m, :][:, l * m:(n - l) * m]
    assert np.abs(inner).max() < 1e-10 * np.abs(T).max() ** 2
    assert np.abs(D).max() > 1e-6


def test_tau_matrix_eigenvalues():
    """H = sqrt(tridiag(-1, 2, -1)) and H_theta of def:matrix_mod_P are diagonalised by S_n
    with eigenvalues eta_j = 2 sin(phi_j / 2), zeta_j."""
    n = 9
    for theta in (1.0, 0.5, 0.3):
        S = sine.dst_matrix(n)
        eta, zeta = pc.ptheta_eigs(n, theta)
        T2 = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        Tt = (theta ** 2 + (1 - theta) ** 2) * np.eye(n) + theta * (1 - theta) * (np.eye(n, k=1) + np.eye(n, k=-1))
        assert np.abs(S @ pc.sqrtm_spd(T2) @ S - np.diag(eta)).max() < 1e-13
        assert np.abs(S @ pc.sqrtm_spd(Tt) @ S - np.diag(zeta)).max() < 1e-13


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_Ptheta_dense_equals_three_steps(theta):
    N, n = 4, 5
    ax, ay = _rand_faces(N, 2, 4)
    s = System(2, N, n, theta=theta, ax=ax, ay=ay, precond="PTHETA")
    P = pc.ptheta_dense(s.K, n, s.tau, theta)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(n * s.m)
    zd = np.linalg.solve(P, v)
    assert np.abs(s.apply_Pinv(v) - zd).max() < 1e-12 * np.abs(zd).max()


def test_chebyshev_is_fixed_spd_polynomial_and_converges():
    """The k-step Chebyshev per-mode operator is linear, symmetric, positive definite,
    and tends to the exact P_theta^{-1} as k grows (error ~ Chebyshev rate)."""
    N, n = 5, 4
    ax, ay = _rand_faces(N, 2, 5, 0.5, 1.5)
    ex = System(2, N, n, theta=1.0, ax=ax, ay=ay, precond="PTHETA")
    M = n * ex.m
    E = np.eye(M)
    Pex = np.column_stack([ex.apply_Pinv(E[:, i]) for i in range(M)])
    prev = np.inf
    for k in (2, 3, 5, 8):
        ch = System(2, N, n, theta=1.0, ax=ax, ay=ay, precond="PTHETA_CHEB", cheb_k=k)
        C = np.column_stack([ch.apply_Pinv(E[:, i]) for i in range(M)])
        assert np.abs(C - C.T).max() < 1e-12 * np.abs(C).max()
        assert np.linalg.eigvalsh(0.5 * (C + C.T)).min() > 0
        err = np.linalg.norm(C - Pex, 2) / np.linalg.norm(Pex, 2)
        assert err < prev
        prev = err
    assert prev < 1e-4


def test_chebyshev_degenerate_interval_is_exact():
    """Constant face values: B_j = A_j, the interval collapses and one application of
    B_j^{-1} is the exact per-mode solve."""
    N, n = 5, 4
    ax, ay = spatial.const_faces(N, 2, 0.7)
    ch = System(2, N, n, theta=0.5, ax=ax, ay=ay, precond="PTHETA_CHEB", cheb_k=3)
    ex = System(2, N, n, theta=0.5, ax=ax, ay=ay, precond="PTHETA")
    v = np.random.default_rng(6).standard_normal(n * ch.m)
    assert np.abs(ch.apply_Pinv(v) - ex.apply_Pinv(v)).max() < 1e-12 * np.abs(ex.apply_Pinv(v)).max()


def test_chebyshev_two_steps_closed_form():
    """k = 2 gives x = (2/c) B^{-1} r - (2/(2c^2 - d^2)) ... written out: with
    c = (hi+lo)/2, d = (hi-lo)/2 the Chebyshev polynomial of degree 1 is
    p(l) = (4c - 2l)/(2c^2 - d^2), i.e. x = p(B^{-1}A) B^{-1} r."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((6, 6))
    A = A @ A.T + 6 * np.eye(6)
    B = np.diag(np.diag(A))
    w = np.linalg.eigvals(np.linalg.solve(B, A)).real
    lo, hi = w.min(), w.max()
    r = rng.standard_normal(6)
    x = pc.chebyshev(lambda z: A @ z, lambda z: np.linalg.solve(B, z), r, 2, lo, hi)
    c, d = 0.5 * (hi + lo), 0.5 * (hi - lo)
    G = np.linalg.solve(B, A)
    P = (4 * c * np.eye(6) - 2 * G) / (2 * c * c - d * d)
    assert np.abs(x - P @ np.linalg.solve(B, r)).max() < 1e-12 * np.abs(x).max()
