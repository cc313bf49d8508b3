"""Pins of the oracle MINRES: the paper's printed iteration counts and errors
(Sec. 5, Tables 1-5), the defining minimal-residual property checked by brute
force, and SciPy's independent MINRES."""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import sine
from oracle.minres import minres
from oracle.system import System

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


@pytest.mark.parametrize("row", _rows("paper_iterations.txt"), ids=lambda r: "-".join(r))
def test_paper_iteration_counts(row):
    tab, ex, theta, n, L, prec, iters = row
    N, n, theta = int(L) - 1, int(n), float(theta)
    p = W.example1(N, n, theta) if ex == "1" else W.example2(N, n, theta)
    s = System(2, N, n, theta=theta, ax=p.ax, ay=p.ay, precond=prec)
    r = s.solve(s.rhs(p.f, p.u0), rtol=1e-6)
    assert r.status == "converged"
    assert r.iters == int(iters), (row, r.iters)


@pytest.mark.parametrize("row", _rows("paper_errors.txt"), ids=lambda r: "-".join(r))
def test_paper_example2_errors(row):
    scheme, n, L, err = row
    N, n, theta = int(L) - 1, int(n), (1.0 if scheme == "BE" else 0.5)
    p = W.example2(N, n, theta)
    s = System(2, N, n, theta=theta, ax=p.ax, ay=p.ay)
    r = s.solve(s.rhs(p.f, p.u0), rtol=1e-6)
    e = np.abs(r.x - W.example2_exact(N, n).reshape(-1)).max()
    # printed to 3 significant digits; the CN values also carry the stopping error
    tol = 0.006 if scheme == "BE" else 0.03
    assert abs(e - float(err)) <= tol * float(err), (e, err)


def test_backward_euler_error_closed_form():
    """As a -> 0 the Example 2 backward-Euler error tends to
    (1/16)(1 - e^{-1})(1 - tau/(e^tau - 1)): the scalar ODE error at the centre node."""
    for n, printed in ((32, 6.14e-4), (64, 3.08e-4)):
        tau = 1.0 / n
        closed = (1 / 16) * (1 - math.exp(-1)) * (1 - tau / (math.exp(tau) - 1))
        assert abs(closed - printed) < 0.006 * printed


def _krylov_min_residual(A, Pinv, b, k):
    """Brute force: minimise ||b - A x||_{P^{-1}} over x in K_k(P^{-1} A, P^{-1} b)."""
    n = len(b)
    V = np.zeros((n, k))
    v = Pinv @ b
    for i in range(k):
        V[:, i] = v
        v = Pinv @ (A @ v)
    Q, _ = np.linalg.qr(V)
    L = np.linalg.cholesky(Pinv)          # Pinv = L L^T, ||r||_{P^{-1}} = ||L^T r||
    M = L.T @ A @ Q
    y, *_ = np.linalg.lstsq(M, L.T @ b, rcond=None)
    return Q @ y


@pytest.mark.parametrize("scheme,theta", [("theta", 1.0), ("theta", 0.5), ("bdf2", 1.0)])
def test_minres_iterates_are_krylov_minimisers(scheme, theta):
    N, n = 3, 6
    rng = np.random.default_rng(11)
    s = System(1, N, n, scheme=scheme, theta=theta)
    A = np.column_stack([s.apply_YT(e) for e in np.eye(n * N)])
    Pinv = np.column_stack([s.apply_Pinv(e) for e in np.eye(n * N)])
    b = rng.standard_normal(n * N)
    for k in (1, 2, 4, 7):
        r = minres(s.apply_YT, s.apply_Pinv, b, rtol=1e-300, maxit=k)
        assert r.iters == k
        xb = _krylov_min_residual(A, Pinv, b, k)
        assert np.abs(r.x - xb).max() < 1e-9 * np.abs(xb).max()


def test_minres_matches_scipy_minres():
    N, n = 7, 16
    p = W.crank_nicolson_2d_noisy(N=N, n=n)
    s = System(2, N, n, theta=0.5)
    rhs = s.flip(s.rhs(p.f, p.u0))
    M = spla.LinearOperator((len(rhs),) * 2, dtype=np.float64,
                            matvec=lambda x: s.apply_Pinv(np.ravel(x).astype(np.float64)))
    A = spla.LinearOperator((len(rhs),) * 2, dtype=np.float64,
                            matvec=lambda x: s.apply_YT(np.ravel(x).astype(np.float64)))
    for k in (3, 6, 9):
        ours = minres(s.apply_YT, s.apply_Pinv, rhs, rtol=1e-300, maxit=k)
        theirs, _ = spla.minres(A, rhs, M=M, maxiter=k, rtol=1e-300)
        assert np.abs(ours.x - theirs).max() < 1e-10 * np.abs(theirs).max()


@pytest.mark.parametrize("precond", ["PH", "PTHETA", "PTHETA_CHEB"])
def test_minres_converges_to_direct_solution(precond):
    N, n = 7, 16
    p = W.variable_coef_2d(N=N, n=n)
    s = System(2, N, n, theta=1.0, ax=p.ax, ay=p.ay, precond=precond, cheb_k=3)
    fH = s.rhs(p.f, p.u0)
    r = s.solve(fH, rtol=1e-12, maxit=200)
    u = s.solve_direct(fH)
    assert r.status == "converged"
    assert np.abs(r.x - u).max() <= 1e-10 * np.abs(u).max()
    assert np.linalg.norm(fH - s.apply_T(r.x)) <= 1e-12 * np.linalg.norm(fH)


def test_minres_warm_start_and_zero_rhs():
    N, n = 5, 8
    s = System(1, N, n, theta=0.5)
    rng = np.random.default_rng(2)
    fH = rng.standard_normal(n * N)
    u = s.solve_direct(fH)
    r = s.solve(fH, rtol=1e-8, x0=u)
    assert r.iters == 0 and r.status == "converged"
    r0 = s.solve(np.zeros(n * N))
    assert r0.iters == 0 and np.all(r0.x == 0)


def test_bdf2_iteration_counts_grow_slowly_with_n():
    """thm:absP_main_gen: the number of outlying eigenvalues is bounded independently
    of n, so the MINRES count grows far slower than n (16x more steps, < 2x iterations)."""
    counts = []
    for n in (16, 64, 256):
        s = System(1, 31, n, scheme="bdf2")
        b = np.random.default_rng(n).standard_normal(n * 31)
        counts.append(s.solve(b, rtol=1e-8).iters)
    assert counts[-1] < 2 * counts[0], counts
