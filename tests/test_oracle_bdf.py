"""Oracle pins for the general BDF-l all-at-once systems of Sec. 4 (l = 3, 4).

The paper leaves the blocks A_(k) of eqn:matrix_gen to the scheme; the oracle takes the
l-step backward difference formula (M = I, multiplied by tau, K only in A_(0)).  The pins:
  * the coefficients reproduce tau u' exactly on polynomials of degree <= l and not l + 1
    (the defining order conditions);
  * a manufactured solution converges at the observed order l in time;
  * Y That is symmetric, That^T = Y That Y;
  * Phat of def:matrix_P_gen, assembled densely from the qbar polynomials and a matrix square
    root, equals the three-step sine-transform form the oracle applies;
  * lemma:rankC_P_gen: That^T That - Phat^2 lives in the first and last l m rows/columns;
  * thm:absC_gen: sqrt(That^T That)^{-1} Y That has eigenvalues +-1 only;
  * MINRES reaches the direct solution and its iterates are the Krylov minimisers.
"""
import math

import numpy as np
import pytest

from oracle import allatonce as aao
from oracle import precond as pc
from oracle.system import System

SCHEMES = [("bdf3", 3), ("bdf4", 4)]


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_bdf_coefficients_order_conditions(l):
    """sum_k alpha_k u(t - k tau) = tau u'(t) for u = 1, t, ..., t^l, but not t^(l+1)."""
    a = aao.bdf_coefficients(l)
    assert len(a) == l + 1
    k = np.arange(l + 1, dtype=np.float64)
    for p in range(l + 1):
        # u(t) = t^p at t = 0: u(-k tau) = (-k tau)^p, tau u'(0) = tau [p == 1]
        lhs = float(np.sum(a * (-k) ** p)) if p > 0 else float(np.sum(a))
        assert abs(lhs - (1.0 if p == 1 else 0.0)) < 1e-13, (l, p, lhs)
    assert abs(float(np.sum(a * (-k) ** (l + 1)))) > 1e-3


def test_bdf2_general_form_equals_the_named_blocks():
    s = System(1, 7, 6, scheme="bdf2")
    g = aao.bdf_blocks(s.K, s.tau, 2)
    for A, B in zip(s.blocks, g):
        assert abs(A - B).max() < 1e-15
    assert np.abs(pc.Phat_dense(s.blocks, 6) - pc.Phat_dense_general(s.blocks, 6)).max() < 1e-12


@pytest.mark.parametrize("scheme,l", SCHEMES)
def test_manufactured_order_in_time(scheme, l):
    """1D, a = 1, f = (1 + pi^2) sin(pi x) e^t: sin(pi x_i) is an exact eigenvector of the
    discrete K (eigenvalue mu_1), so the semi-discrete solution is c(t) sin(pi x_i) with
    c' = -mu_1 c + (1 + pi^2) e^t, c(0) = 1, i.e. c(t) = B e^t + (1 - B) e^{-mu_1 t},
    B = (1 + pi^2)/(1 + mu_1).  With the exact history values c(t_0), c(t_{-1}), ... moved to
    the right-hand side, the all-at-once BDF-l solution must approach it at order l."""
    N = 7
    errs = []
    for n in (32, 64, 128):
        s = System(1, N, n, scheme=scheme)
        tau = s.tau
        x = np.arange(1, N + 1) / (N + 1)
        mu1 = 4.0 * (N + 1) ** 2 * math.sin(math.pi / (2 * (N + 1))) ** 2
        B = (1 + math.pi ** 2) / (1 + mu1)
        c = lambda t: B * math.exp(t) + (1 - B) * math.exp(-mu1 * t)
        a = s.alpha
        b = np.zeros((n, N))
        for k in range(1, n + 1):
            b[k - 1] = tau * (1 + math.pi ** 2) * math.exp(k * tau) * np.sin(math.pi * x)
            for j in range(k, l + 1):              # history levels t_{k-j} <= 0
                b[k - 1] -= a[j] * c((k - j) * tau) * np.sin(math.pi * x)
        u = s.solve_direct(b.reshape(-1)).reshape(n, N)
        exact = np.array([c(k * tau) for k in range(1, n + 1)])[:, None] * np.sin(math.pi * x)[None, :]
        errs.append(np.abs(u - exact).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(orders[-1] - l) < 0.3, (errs, orders)


@pytest.mark.parametrize("scheme,l", SCHEMES)
def test_YT_symmetric_and_transpose(scheme, l):
    N, n = 3, 9
    rng = np.random.default_rng(41)
    ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
    s = System(2, N, n, scheme=scheme, ax=ax, ay=ay)
    T = s.assemble_T().toarray()
    Y = aao.flip(n, s.m).toarray()
    assert np.abs(Y @ T - (Y @ T).T).max() == 0.0
    assert np.abs(T.T - Y @ T @ Y).max() == 0.0
    x = rng.standard_normal(n * s.m)
    assert np.abs(s.apply_YT(x) - Y @ T @ x).max() < 1e-12 * np.abs(T).max()
    fH = rng.standard_normal(n * s.m)
    assert np.abs(s.solve_direct(fH) - np.linalg.solve(T, fH)).max() < 1e-11 * np.abs(np.linalg.solve(T, fH)).max()


@pytest.mark.parametrize("scheme,l", SCHEMES)
def test_Phat_dense_equals_dst_form(scheme, l):
    """def:matrix_P_gen through qbar_0..qbar_l and a dense matrix square root equals the
    three-step form (time and space sine transforms, division by |ghat(phi_j)|)."""
    for dim, N, n, kind in ((1, 5, 8, "const"), (2, 3, 7, "var")):
        ax = ay = None
        if kind == "var":
            rng = np.random.default_rng(42)
            ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
        s = System(dim, N, n, scheme=scheme, ax=ax, ay=ay)
        if kind == "const":
            blocks = s.blocks
        else:   # variable a: P uses the averaged Kbar of Sec. 3.1.1 in place of K
            from oracle import spatial
            blocks = aao.bdf_blocks(spatial.kbar_matrix(N, dim, ax, ay), s.tau, l)
        Ph = pc.Phat_dense_general(blocks, n)
        v = np.random.default_rng(43).standard_normal(n * s.m)
        ref = np.linalg.solve(Ph, v)
        assert np.abs(s.apply_Pinv(v) - ref).max() < 1e-12 * np.abs(ref).max(), (dim, kind)


@pytest.mark.parametrize("scheme,l", SCHEMES)
def test_corner_structure_lemma(scheme, l):
    """lemma:rankC_P_gen: That^T That - Phat^2 vanishes outside the first and last l m
    rows and columns (and is not zero)."""
    N, n = 3, 4 * 4 + 3
    s = System(1, N, n, scheme=scheme)
    Ph = pc.Phat_dense_general(s.blocks, n)
    T = s.assemble_T().toarray()
    D = T.T @ T - Ph @ Ph
    m = s.m
    inner = D[l * m:(n - l) * m, :][:, l * m:(n - l) * m]
    assert np.abs(inner).max() < 1e-10 * np.abs(T).max() ** 2
    # the nonzero part sits in the two corners: rows past l m that reach past l m columns vanish
    assert np.abs(D[l * m:(n - l) * m, :]).max() < 1e-10 * np.abs(T).max() ** 2
    assert np.abs(D).max() > 1e-6


@pytest.mark.parametrize("scheme,l", SCHEMES)
def test_abs_preconditioner_eigs_pm1(scheme, l):
    N, n = 3, 6
    s = System(2, N, n, scheme=scheme)
    T = s.assemble_T().toarray()
    Y = aao.flip(n, s.m).toarray()
    Q = np.linalg.solve(pc.sqrtm_spd(T.T @ T), Y @ T)
    assert np.abs(Q - Q.T).max() < 1e-10
    assert np.abs(Q @ Q.T - np.eye(len(Q))).max() < 1e-10
    ev = np.linalg.eigvals(Q)
    assert np.abs(np.abs(ev.real) - 1).max() < 1e-9 and np.abs(ev.imag).max() < 1e-9


@pytest.mark.parametrize("scheme,l", SCHEMES)
def test_minres_reaches_direct_solution_and_krylov_minimiser(scheme, l):
    """The preconditioned MINRES iterate minimises ||P^{-1/2}(b - A x)|| over the Krylov
    space of P^{-1} A (checked by a dense least-squares solve after 3 steps) and the solve
    reaches the direct solution."""
    N, n = 7, 24
    rng = np.random.default_rng(44)
    ax, ay = rng.uniform(0.5, 1.5, (N, N + 1)), rng.uniform(0.5, 1.5, (N + 1, N))
    s = System(2, N, n, scheme=scheme, ax=ax, ay=ay)
    b = rng.standard_normal(n * s.m)
    r = s.solve(b, rtol=1e-10, maxit=400)
    u = s.solve_direct(b)
    assert r.status == "converged"
    assert np.abs(r.x - u).max() < 1e-7 * np.abs(u).max()
    # Krylov minimiser after k steps in the P^{-1} norm of the residual
    k = 3
    rk = s.solve(b, rtol=1e-300, maxit=k)
    A = lambda x: s.apply_YT(x)
    rhs = s.flip(b)
    Pinv = s.apply_Pinv
    z = Pinv(rhs)
    V = [z]
    for _ in range(k - 1):
        V.append(Pinv(A(V[-1])))
    V = np.stack(V, axis=1)
    AV = np.stack([A(V[:, i]) for i in range(k)], axis=1)
    # minimise (rhs - AV c)^T P^{-1} (rhs - AV c): P^{-1/2} via the dense Phat
    G = np.stack([Pinv(AV[:, i]) for i in range(k)], axis=1)
    M = AV.T @ G
    c = np.linalg.solve(0.5 * (M + M.T), G.T @ rhs)
    xk = V @ c
    assert np.abs(rk.x - xk).max() < 1e-8 * np.abs(xk).max()
