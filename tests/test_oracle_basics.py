"""Pins of the oracle's building blocks against closed forms and independent constructions.

Every check here is against something other than the oracle's own formula: the
closed-form DST-I eigenpairs, SciPy's FFT-based DST, the energy form
K = D^T diag(a) D / h^2, dense eigen-decompositions, and plain time stepping.
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp

import workloads as W
from oracle import allatonce as aao
from oracle import precond as pc
from oracle import sine, spatial
from oracle.system import System


# ---------------------------------------------------------------- sine transform (Sec. 3.1.1)

@pytest.mark.parametrize("n", [1, 2, 5, 6, 16, 31])
def test_dst_matrix_orthogonal_involutory(n):
    S = sine.dst_matrix(n)
    assert np.allclose(S, S.T, atol=0, rtol=0) or np.abs(S - S.T).max() < 1e-15
    assert np.abs(S @ S - np.eye(n)).max() < 1e-14


@pytest.mark.parametrize("n", [3, 6, 17])
def test_dst_diagonalises_Pn(n):
    S = sine.dst_matrix(n)
    D = S @ sine.tridiag_half(n) @ S
    assert np.abs(D - np.diag(sine.cos_phi(n))).max() < 1e-14


@pytest.mark.parametrize("n", [4, 7, 64])
def test_dst_dense_equals_scipy_fft(n):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, 3))
    assert np.abs(sine.dst_matrix(n) @ x - scipy.fft.dst(x, type=1, norm="ortho", axis=0)).max() < 1e-13


# ---------------------------------------------------------------- stiffness matrix (eqn:matrix_Km_va)

@pytest.mark.parametrize("dim,N", [(1, 1), (1, 9), (2, 1), (2, 5), (2, 8)])
def test_stiffness_equals_energy_form(dim, N):
    rng = np.random.default_rng(1)
    if dim == 1:
        ax, ay = rng.uniform(0.5, 2.0, N + 1), None
    else:
        ax, ay = rng.uniform(0.5, 2.0, (N, N + 1)), rng.uniform(0.5, 2.0, (N + 1, N))
    K = spatial.stiffness(N, dim, ax, ay).toarray()
    Dx, Dy = spatial.face_difference(N, dim)
    E = Dx.T @ sp.diags(np.ravel(ax)) @ Dx
    if dim == 2:
        E = E + Dy.T @ sp.diags(np.ravel(ay)) @ Dy
    E = E.toarray() * (N + 1) ** 2
    assert np.abs(K - E).max() <= 1e-12 * np.abs(E).max()
    assert np.abs(K - K.T).max() == 0.0
    assert np.linalg.eigvalsh(K).min() > 0


@pytest.mark.parametrize("dim,N", [(1, 7), (2, 7)])
def test_constant_coefficient_eigenpairs(dim, N):
    """K(1) = U diag(mu) U with U = S_N or S_N (x) S_N and mu the closed form."""
    K = spatial.stiffness(N, dim).toarray()
    S = sine.dst_matrix(N)
    U = S if dim == 1 else np.kron(S, S)
    mu = spatial.mu_const(N, dim)
    assert np.abs(U @ K @ U - np.diag(mu)).max() < 1e-10 * mu.max()
    assert np.abs(np.sort(mu) - np.linalg.eigvalsh(K)).max() < 1e-10 * mu.max()


def test_kbar_literal_average_and_eigs():
    N = 6
    rng = np.random.default_rng(2)
    ax, ay = rng.uniform(0.5, 2.0, (N, N + 1)), rng.uniform(0.5, 2.0, (N + 1, N))
    K = spatial.stiffness(N, 2, ax, ay).toarray()
    h2 = (1.0 / (N + 1)) ** 2
    d, cx, cy = spatial.kbar_params(N, 2, ax, ay)
    # literal averages of K's diagonal and of its nonzero +-1 and +-N couplings
    assert abs(d - np.mean(np.diag(K)) * h2) < 1e-12
    xc = np.array([K[j * N + i, j * N + i + 1] for j in range(N) for i in range(N - 1)])
    yc = np.array([K[j * N + i, (j + 1) * N + i] for j in range(N - 1) for i in range(N)])
    assert abs(cx + np.mean(xc) * h2) < 1e-12
    assert abs(cy + np.mean(yc) * h2) < 1e-12
    Kb = spatial.kbar_matrix(N, 2, ax, ay).toarray()
    S = sine.dst_matrix(N)
    U = np.kron(S, S)
    mu = spatial.mu_kbar(N, 2, ax, ay)
    assert np.abs(U @ Kb @ U - np.diag(mu)).max() < 1e-10 * np.abs(mu).max()


def test_kbar_literal_can_be_indefinite():
    """Reading of the averaging: the literal average can lose definiteness
    (1D, a = 1 + sin(pi x)); P_H(Kbar) stays SPD because it uses moduli."""
    N = 15
    ax, _ = W.sample_faces(lambda x: 1.0 + np.sin(np.pi * x), N, 1)
    mu = spatial.mu_kbar(N, 1, ax)
    assert mu.min() < 0
    sig = pc.sigma_theta(mu, 8, 1.0 / 8, 1.0)
    assert sig.min() > 0


def test_faces_from_nodal():
    N = 4
    a = W.sample_nodal(lambda x, y: 1 + x + 10 * y, N, 2)
    ax, ay = spatial.faces_from_nodal(a, 2)
    bx, by = W.sample_faces(lambda x, y: 1 + x + 10 * y, N, 2)
    # linear a: mean of the endpoint nodes equals the midpoint value
    assert np.abs(ax - bx).max() < 1e-13 and np.abs(ay - by).max() < 1e-13


# ---------------------------------------------------------------- all-at-once system (eq. theta, eqn:matrix_gen)

@pytest.mark.parametrize("scheme,theta", [("theta", 1.0), ("theta", 0.5), ("theta", 0.3), ("bdf2", 1.0)])
def test_YT_symmetric_and_transpose_identity(scheme, theta):
    N, n = 4, 6
    rng = np.random.default_rng(3)
    ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
    s = System(2, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay)
    T = s.assemble_T().toarray()
    Y = aao.flip(n, s.m).toarray()
    assert np.abs(Y @ T - (Y @ T).T).max() == 0.0
    assert np.abs(T.T - Y @ T @ Y).max() == 0.0
    x = rng.standard_normal(n * s.m)
    assert np.abs(s.apply_YT(x) - Y @ T @ x).max() < 1e-12 * np.abs(T).max()


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.25])
def test_allatonce_equals_time_stepping(theta):
    N, n = 6, 9
    rng = np.random.default_rng(4)
    ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
    s = System(2, N, n, theta=theta, ax=ax, ay=ay)
    f = rng.standard_normal((n + 1, s.m))
    u0 = rng.standard_normal(s.m)
    fH = s.rhs(f, u0)
    u_seq = aao.sequential_theta_steps(f, u0, s.K, s.tau, theta)
    u_all = s.solve_direct(fH)
    u_dense = np.linalg.solve(s.assemble_T().toarray(), fH)
    assert np.abs(u_all - u_seq).max() <= 1e-12 * np.abs(u_seq).max()
    assert np.abs(u_dense - u_seq).max() <= 1e-12 * np.abs(u_seq).max()
    # brute force on the permuted symmetric system
    Y = aao.flip(n, s.m).toarray()
    u_sym = np.linalg.solve(Y @ s.assemble_T().toarray(), Y @ fH)
    assert np.abs(u_sym - u_seq).max() <= 1e-12 * np.abs(u_seq).max()


def test_bdf2_direct_matches_recursion():
    N, n = 5, 8
    rng = np.random.default_rng(6)
    s = System(1, N, n, scheme="bdf2")
    b = rng.standard_normal((n, N))
    u = s.solve_direct(b.reshape(-1)).reshape(n, N)
    A0 = (1.5 * np.eye(N) + s.tau * s.K.toarray())
    up, upp = np.zeros(N), np.zeros(N)
    for k in range(n):
        uk = np.linalg.solve(A0, b[k] + 2 * up - 0.5 * upp)
        assert np.abs(uk - u[k]).max() < 1e-12 * max(1, np.abs(uk).max())
        upp, up = up, uk


def test_manufactured_1d_scalar_recurrence():
    """sin(pi x_i) is an exact eigenvector of the discrete K, so the backward-Euler
    solution is c_k sin(pi x_i) with (1 + tau mu_1) c_k = c_{k-1} + tau (1 + pi^2) e^{t_k}."""
    p = W.manufactured_1d(N=63, n=64)
    s = System(1, p.N, p.n, theta=1.0)
    u = s.solve_direct(s.rhs(p.f, p.u0)).reshape(p.n, p.N)
    mu1 = 4 * (p.N + 1) ** 2 * math.sin(math.pi / (2 * (p.N + 1))) ** 2
    c = 1.0
    xi = W.interior(p.N)
    for k in range(1, p.n + 1):
        c = (c + p.tau * (1 + math.pi ** 2) * math.exp(k * p.tau)) / (1 + p.tau * mu1)
        assert np.abs(u[k - 1] - c * np.sin(math.pi * xi)).max() < 1e-12 * c


@pytest.mark.parametrize("theta,order", [(1.0, 1.0), (0.5, 2.0)])
def test_manufactured_time_order(theta, order):
    """Against the exact solution of the semi-discrete ODE c' = -mu_1 c + (1 + pi^2) e^t
    (sin(pi x_i) is an eigenvector of K), the time error falls like tau (backward
    Euler) or tau^2 (Crank-Nicolson)."""
    N = 63
    mu = 4 * (N + 1) ** 2 * math.sin(math.pi / (2 * (N + 1))) ** 2
    xi = W.interior(N)
    errs = []
    for n in (16, 32, 64):
        p = W.manufactured_1d(N=N, n=n, theta=theta)
        s = System(1, N, n, theta=theta)
        u = s.solve_direct(s.rhs(p.f, p.u0)).reshape(n, N)
        t = np.arange(1, n + 1) / n
        c = np.exp(-mu * t) + (1 + math.pi ** 2) * (np.exp(t) - np.exp(-mu * t)) / (1 + mu)
        errs.append(np.abs(u - c[:, None] * np.sin(math.pi * xi)[None, :]).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - order) < 0.15 for r in rates), rates


def test_space_order():
    errs = []
    for N in (15, 31, 63):
        p = W.manufactured_1d(N=N, n=2048, theta=0.5)
        s = System(1, N, 2048, theta=0.5)
        u = s.solve_direct(s.rhs(p.f, p.u0)).reshape(2048, N)
        errs.append(np.abs(u[-1] - np.sin(math.pi * W.interior(N)) * math.e).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - 2.0) < 0.15 for r in rates), rates
