"""Pins of the adjoint solve and the gradients: dense T^{-T}, the dot-product
test, and central finite differences on direct (sequential) solves."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import spatial
from oracle.system import System


def _loss_and_grads(theta, N=4, n=5, dim=2, seed=0):
    rng = np.random.default_rng(seed)
    a_nodal = rng.uniform(0.7, 1.3, (N + 2,) * dim)
    f = rng.standard_normal((n + 1, N ** dim))
    u0 = rng.standard_normal(N ** dim)
    uobs = rng.standard_normal(n * N ** dim)

    def loss(a_nodal, f, u0):
        s = System(dim, N, n, theta=theta, a_nodal=a_nodal)
        u = s.solve_direct(s.rhs(f, u0))
        return float(np.sum((u - uobs) ** 2)), s, u

    L, s, u = loss(a_nodal, f, u0)
    g = 2 * (u - uobs)
    lam = adj.adjoint_dense(s, g)
    gf, gu0 = adj.rhs_adjoint(s, lam)
    gx, gy = adj.grad_faces(s, u, u0, lam)
    gn = adj.grad_nodal(gx, gy, N, dim)
    return loss, (a_nodal, f, u0), (gf, gu0, gx, gy, gn), s, lam, g


def test_adjoint_identity_and_minres_adjoint():
    """T^T = Y T Y: MINRES on (Y T) mu = g then lambda = Y mu solves T^T lambda = g."""
    N, n = 4, 6
    rng = np.random.default_rng(1)
    ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
    s = System(2, N, n, theta=0.5, ax=ax, ay=ay)
    g = rng.standard_normal(n * s.m)
    lam, res = adj.adjoint_solve(s, g, rtol=1e-13)
    lam_d = adj.adjoint_dense(s, g)
    assert np.abs(lam - lam_d).max() < 1e-10 * np.abs(lam_d).max()
    x = rng.standard_normal(n * s.m)
    T = s.assemble_T()
    assert abs((T @ x) @ lam_d - x @ g) < 1e-10 * abs(x @ g)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_gradients_against_central_differences(theta):
    loss, (a, f, u0), (gf, gu0, gx, gy, gn), s, lam, g = _loss_and_grads(theta)
    rng = np.random.default_rng(9)
    h = 1e-6
    # nodal a
    d = rng.standard_normal(a.shape)
    fd = (loss(a + h * d, f, u0)[0] - loss(a - h * d, f, u0)[0]) / (2 * h)
    assert abs(fd - np.sum(gn * d)) <= 1e-6 * max(1.0, abs(fd))
    # f, all levels k = 0..n
    d = rng.standard_normal(f.shape)
    fd = (loss(a, f + h * d, u0)[0] - loss(a, f - h * d, u0)[0]) / (2 * h)
    assert abs(fd - np.sum(gf * d)) <= 1e-6 * max(1.0, abs(fd))
    # u0
    d = rng.standard_normal(u0.shape)
    fd = (loss(a, f, u0 + h * d)[0] - loss(a, f, u0 - h * d)[0]) / (2 * h)
    assert abs(fd - np.sum(gu0 * d)) <= 1e-6 * max(1.0, abs(fd))


def test_face_gradient_against_central_differences():
    theta, N, n = 0.5, 4, 5
    rng = np.random.default_rng(3)
    ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
    f = rng.standard_normal((n + 1, N * N))
    u0 = rng.standard_normal(N * N)
    w = rng.standard_normal(n * N * N)

    def loss(ax, ay):
        s = System(2, N, n, theta=theta, ax=ax, ay=ay)
        return float(w @ s.solve_direct(s.rhs(f, u0))), s

    L, s = loss(ax, ay)
    u = s.solve_direct(s.rhs(f, u0))
    lam = adj.adjoint_dense(s, w)
    gx, gy = adj.grad_faces(s, u, u0, lam)
    dx, dy = rng.standard_normal(ax.shape), rng.standard_normal(ay.shape)
    h = 1e-6
    fd = (loss(ax + h * dx, ay + h * dy)[0] - loss(ax - h * dx, ay - h * dy)[0]) / (2 * h)
    assert abs(fd - np.sum(gx * dx) - np.sum(gy * dy)) <= 1e-6 * max(1.0, abs(fd))


def test_nodal_gradient_is_face_scatter():
    N = 3
    rng = np.random.default_rng(4)
    gx, gy = rng.standard_normal((N, N + 1)), rng.standard_normal((N + 1, N))
    gn = adj.grad_nodal(gx, gy, N, 2)
    # <gn, da> must equal <g_faces, d faces> for every nodal perturbation da
    da = rng.standard_normal((N + 2, N + 2))
    fx, fy = spatial.faces_from_nodal(da, 2)
    assert abs(np.sum(gn * da) - np.sum(gx * fx) - np.sum(gy * fy)) < 1e-12


def test_adjoint_direct_matches_dense():
    for scheme, theta in (("theta", 0.5), ("theta", 1.0), ("bdf2", 1.0)):
        N, n = 4, 7
        rng = np.random.default_rng(5)
        ax, ay = rng.uniform(0.5, 2, (N, N + 1)), rng.uniform(0.5, 2, (N + 1, N))
        s = System(2, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay)
        g = rng.standard_normal(n * s.m)
        ld = adj.adjoint_dense(s, g)
        assert np.abs(adj.adjoint_direct(s, g) - ld).max() < 1e-12 * np.abs(ld).max()
