"""Iterate parity at the shapes the full-size workloads launch.

The fused sine-basis kernel pads the folded time halves to hp = next power of two of
ceil(n/2) and picks its matrix-core tiling from hp; the batched launch groups instances by
hp; the physical-basis path picks its time-transform and spatial-transform kernels from hp
and N + 1.  These tests drive every such instantiation that a shipped workload reaches
(hp = 128 at both column-tile widths, hp = 256 and 512 on the fused and the physical path,
the hp = 128 class of a batch, N + 1 = 256 on the physical path) and the full 2D
Crank-Nicolson workload itself, and require what Sec. 5's experiments fix: from x0 = 0 the
GPU stops at the oracle's iteration (first true relative residual <= rtol) and its iterate
equals the oracle's to 1e-10 relative (max norm)."""
import numpy as np
import pytest

import workloads as W
from oracle.system import System

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)).to(_dev())


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _smooth_faces(N):
    return W.sample_faces(lambda x, y: 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y), N, 2)


def _rhs(o, scheme, n, m, seed):
    rng = np.random.default_rng(seed)
    if scheme == "theta":
        return o.rhs(rng.standard_normal((n + 1, m)), rng.standard_normal(m))
    return rng.standard_normal(n * m)


def _check(g, o, b, rtol=1e-8, maxit=400):
    ref = o.solve(b, rtol=rtol, maxit=maxit)
    x, info = g.solve(_t(b), rtol=rtol, maxit=maxit)
    x = _n(x)
    assert ref.status == "converged" and info["status"] == "ok", (info, ref.status)
    assert info["iters"] == ref.iters, (info["iters"], ref.iters)
    assert rel(x, ref.x) < 1e-10
    assert info["relres_true"] <= rtol
    return info, ref


def test_cn2d_full_size_iterate_parity():
    """The 2D Crank-Nicolson workload at full size (N = 127, n = 256, noisy source, seed 0):
    the headline fused kernel k_spec<128, 32> with the width chosen at setup."""
    from paper_2201_10062_amd import Plan
    _dev()
    p = W.crank_nicolson_2d_noisy()
    g = Plan(2, p.N, p.n, theta=0.5)
    o = System(2, p.N, p.n, theta=0.5)
    b = o.rhs(p.f, p.u0)
    info, ref = _check(g, o, b)
    print(f"cn2d full: iters {info['iters']} (oracle {ref.iters}) relres {info['relres_true']:.6e} "
          f"(oracle {ref.relres_true:.6e}) width {g.tile_cols}")
    assert abs(info["relres_true"] - ref.relres_true) <= 1e-6 * ref.relres_true


@pytest.mark.parametrize("cols", [16, 32])
@pytest.mark.parametrize("n", [200, 256])
@pytest.mark.parametrize("scheme,theta,kind", [("theta", 0.5, "const"), ("bdf2", 1.0, "const"),
                                               ("theta", 1.0, "smooth"), ("bdf2", 1.0, "smooth")])
def test_fused_hp128_both_widths(scheme, theta, kind, n, cols):
    """hp = 128 (ceil(n/2) in (64, 128]): the matrix-core tiling with two row tiles per wave,
    constant a (time stencil in the fused kernel) and variable a (per-level matvec)."""
    from paper_2201_10062_amd import Plan
    _dev()
    N = 31
    ax, ay = (None, None) if kind == "const" else _smooth_faces(N)
    g = Plan(2, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay, tile_cols=cols)
    assert g.tile_cols == cols
    o = System(2, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay)
    _check(g, o, _rhs(o, scheme, n, g.m, 40 + n))


@pytest.mark.parametrize("n", [300, 600])
@pytest.mark.parametrize("scheme,theta", [("theta", 0.5), ("bdf2", 1.0)])
def test_fused_hp256_hp512(scheme, theta, n):
    """hp = 256 and 512 on the fused kernel (constant a, 16-column tiles only)."""
    from paper_2201_10062_amd import Plan
    _dev()
    N = 15
    g = Plan(2, N, n, scheme=scheme, theta=theta)
    assert g.tile_cols == 16
    o = System(2, N, n, scheme=scheme, theta=theta)
    _check(g, o, _rhs(o, scheme, n, g.m, 50 + n))


def test_batch_with_hp128_class():
    """A batch whose largest time-size class is hp = 128 (n = 200, 256), with constant and
    variable coefficients and the 32-column class the batch chooses; each instance against
    its own oracle."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    probs = W.bdf2_batch(count=12, Ns=(15, 31), ns=(64, 200, 256))
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay) for p in probs]
    assert any(p.n >= 200 for p in probs) and any(p.ax is not None and p.n >= 200 for p in probs)
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], rtol=1e-8)
    for p, x, info in zip(probs, xs, infos):
        o = System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay)
        ref = o.solve(p.b.reshape(-1), rtol=1e-8, maxit=500)
        assert info["status"] == "ok" and info["iters"] == ref.iters, (p.name, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-10, p.name


@pytest.mark.parametrize("precond", ["PH", "PTHETA_CHEB"])
def test_physical_path_hp256(precond):
    """The physical-basis iteration at hp = 256 (n = 300): the time transform with one folded
    block per pass, P_H(Kbar) and P_theta with 3 Chebyshev steps."""
    from paper_2201_10062_amd import Plan
    _dev()
    N, n = 31, 300
    ax, ay = _smooth_faces(N)
    g = Plan(2, N, n, theta=1.0, precond=precond, cheb_k=3, ax=ax, ay=ay, general_path=True)
    assert g.tile_cols == 0
    o = System(2, N, n, theta=1.0, ax=ax, ay=ay, precond=precond, cheb_k=3)
    _check(g, o, _rhs(o, "theta", n, g.m, 60))


@pytest.mark.parametrize("n", [100, 129, 200])
@pytest.mark.parametrize("precond", ["PH", "PTHETA_CHEB"])
def test_physical_path_hp64_hp128(precond, n):
    """The physical-basis time transform at hp = 64 (n = 100) and hp = 128 (n = 129, odd: the
    middle level has no odd-symmetric partner; n = 200), one folded block per pass on four or
    eight matrix-core waves: P^{-1} to 1e-12, and the MINRES iterate to 1e-10 at the oracle's
    stopping iteration, for P_H(Kbar) and P_theta with 3 Chebyshev steps."""
    from paper_2201_10062_amd import Plan
    _dev()
    N = 31
    ax, ay = _smooth_faces(N)
    g = Plan(2, N, n, theta=1.0, precond=precond, cheb_k=3, ax=ax, ay=ay, general_path=True)
    assert g.tile_cols == 0
    o = System(2, N, n, theta=1.0, ax=ax, ay=ay, precond=precond, cheb_k=3)
    v = np.random.default_rng(61).standard_normal(n * g.m)
    assert rel(_n(g.apply_P_inv(_t(v))), o.apply_Pinv(v)) < 1e-12
    _check(g, o, _rhs(o, "theta", n, g.m, 62))


def test_physical_path_hp128_fp32():
    """Float32 time transforms at hp = 128 on the physical path (parity unpinned by rounding):
    the float64 true residual at the tolerance, iterations within 10% (+1) of the oracle's."""
    from paper_2201_10062_amd import Plan
    _dev()
    N, n = 31, 200
    ax, ay = _smooth_faces(N)
    g = Plan(2, N, n, theta=1.0, ax=ax, ay=ay, general_path=True, pprec="fp32")
    o = System(2, N, n, theta=1.0, ax=ax, ay=ay)
    b = _rhs(o, "theta", n, g.m, 63)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    x = _n(x)
    r = np.linalg.norm(b - o.apply_T(x)) / np.linalg.norm(b)
    assert info["status"] == "ok" and r <= 1e-8
    assert info["iters"] <= int(1.1 * ref.iters) + 1
    assert rel(x, ref.x) < 1e-6


@pytest.mark.parametrize("precond", ["PH", "PTHETA_CHEB"])
def test_physical_path_N255_two_iterations(precond):
    """N + 1 = 256 (the persistent 512-point spatial transform) with the variable coefficient
    of the 2D variable-coefficient workload: two MINRES iterations equal the oracle's."""
    from paper_2201_10062_amd import Plan
    _dev()
    p = W.variable_coef_2d(N=255, n=48)
    g = Plan(2, p.N, p.n, theta=1.0, precond=precond, cheb_k=3, ax=p.ax, ay=p.ay)
    assert g.tile_cols == 0
    o = System(2, p.N, p.n, theta=1.0, ax=p.ax, ay=p.ay, precond=precond, cheb_k=3)
    b = o.rhs(p.f, p.u0)
    ref = o.solve(b, rtol=1e-300, maxit=2)
    x, info = g.solve(_t(b), rtol=1e-300, maxit=2, raise_on_fail=False)
    assert info["iters"] == 2 == ref.iters and info["status"] == "enotconv"
    assert rel(_n(x), ref.x) < 1e-10
    assert abs(info["relres_true"] - ref.relres_true) <= 1e-9 * ref.relres_true


def test_fp32_hp128_fused_and_batched():
    """Mixed precision at hp = 128 (parity unpinned by rounding): the float64 true residual
    reaches the tolerance, the iteration count stays within 10% (+1) of the float64 oracle's,
    and the error against the oracle is reported; single plan and batch."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    probs = W.bdf2_batch(count=6, Ns=(31,), ns=(256, 200))
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, pprec="fp32") for p in probs]
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], rtol=1e-8)
    for p, g, x, info in zip(probs, plans, xs, infos):
        o = System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay)
        ref = o.solve(p.b.reshape(-1), rtol=1e-8, maxit=500)
        xb = _n(x)
        r = np.linalg.norm(p.b.reshape(-1) - o.apply_T(xb)) / np.linalg.norm(p.b)
        x1, info1 = g.solve(_t(p.b), rtol=1e-8)
        r1 = np.linalg.norm(p.b.reshape(-1) - o.apply_T(_n(x1))) / np.linalg.norm(p.b)
        print(f"fp32 hp128 {p.name}: batched iters {info['iters']} single {info1['iters']} (fp64 {ref.iters}) "
              f"err {rel(xb, ref.x):.2e}")
        for rr, inf in ((r, info), (r1, info1)):
            assert inf["status"] == "ok" and rr <= 1e-8
            assert inf["iters"] <= int(1.1 * ref.iters) + 1
        assert rel(xb, ref.x) < 1e-6
