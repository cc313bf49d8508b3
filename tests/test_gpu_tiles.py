"""Column-tile width of the fused sine-basis kernel (spatial modes per workgroup).  Either
width, forced, must reproduce the FP64 oracle's MINRES iteration count and iterate (the width
changes only the summation order of the reductions); the width timed at setup is one of the
two; a batch may hold plans of both widths."""
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


def _faces(kind, N, seed=3):
    if kind == "const":
        return None, None
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.5, (N, N + 1)), rng.uniform(0.5, 1.5, (N + 1, N))


CASES = [
    (2, 31, 64, "theta", 0.5, "const"),
    (2, 63, 128, "theta", 1.0, "const"),
    (2, 127, 8, "theta", 1.0, "const"),
    (1, 63, 64, "theta", 1.0, "const"),
    (2, 31, 40, "bdf2", 1.0, "var"),
    (2, 63, 17, "theta", 0.5, "var"),
]


@pytest.mark.parametrize("cols", [16, 32])
@pytest.mark.parametrize("dim,N,n,scheme,theta,kind", CASES)
def test_forced_tile_width_parity(dim, N, n, scheme, theta, kind, cols):
    from paper_2201_10062_amd import Plan
    _dev()
    ax, ay = _faces(kind, N) if dim == 2 else (None, None)
    g = Plan(dim, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay, tile_cols=cols)
    assert g.tile_cols == cols
    o = System(dim, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay)
    rng = np.random.default_rng(5)
    b = o.rhs(rng.standard_normal((n + 1, g.m)), rng.standard_normal(g.m)) if scheme == "theta" \
        else rng.standard_normal(n * g.m)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    assert ref.status == "converged" and info["status"] == "ok"
    assert info["iters"] == ref.iters
    assert rel(_n(x), ref.x) < 1e-10
    assert info["relres_true"] <= 1e-8


def test_fp32_tile_widths():
    """Mixed precision at both widths: the float64 true residual reaches the tolerance and the
    iteration count stays within 10% (+1) of the float64 oracle's."""
    from paper_2201_10062_amd import Plan
    _dev()
    o = System(2, 63, 64, theta=0.5)
    rng = np.random.default_rng(6)
    b = o.rhs(rng.standard_normal((65, 63 * 63)), rng.standard_normal(63 * 63))
    ref = o.solve(b, rtol=1e-8)
    for cols in (16, 32):
        g = Plan(2, 63, 64, theta=0.5, pprec="fp32", tile_cols=cols)
        x, info = g.solve(_t(b), rtol=1e-8)
        r = np.linalg.norm(b - o.apply_T(_n(x))) / np.linalg.norm(b)
        assert info["status"] == "ok" and r <= 1e-8, cols
        assert info["iters"] <= int(1.1 * ref.iters) + 1
        assert rel(_n(x), ref.x) < 1e-6


def test_tuned_width_and_limits():
    from paper_2201_10062_amd import Plan, SmrError
    _dev()
    assert Plan(2, 31, 64).tile_cols in (16, 32)
    assert Plan(2, 63, 64, pprec="fp32").tile_cols in (16, 32)
    assert Plan(2, 15, 512).tile_cols == 16                   # ceil(n/2) > 128: 16 only
    assert Plan(2, 31, 8, general_path=True).tile_cols == 0   # physical basis
    ax, ay = _faces("var", 15)
    assert Plan(2, 15, 8, ax=ax, ay=ay).tile_cols == 0        # N + 1 = 16: physical basis
    with pytest.raises(SmrError):
        Plan(2, 15, 512, tile_cols=32)


def test_batch_mixes_tile_widths():
    """One batch holding plans of the same time padding at both widths (two launch classes);
    solved twice so the second call replays the cached graph; every instance equals the oracle."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    probs = W.bdf2_batch(count=8, Ns=(15, 31), ns=(32, 48))
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, tile_cols=(16, 32)[(i // 2 + i) % 2])
             for i, p in enumerate(probs)]
    refs = [System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay).solve(p.b.reshape(-1), rtol=1e-9, maxit=500)
            for p in probs]
    batch = Batch(plans)
    for rep in range(2):
        xs, infos = batch.solve([_t(p.b) for p in probs], rtol=1e-9)
        for p, x, info, ref in zip(probs, xs, infos, refs):
            assert info["status"] == "ok" and info["iters"] == ref.iters, (rep, p.name, info, ref.iters)
            assert rel(_n(x), ref.x) < 1e-9, (rep, p.name)


@pytest.mark.parametrize("scheme,theta,N,n,pprec", [("theta", 0.5, 63, 64, "fp64"), ("bdf4", 1.0, 127, 40, "fp64"),
                                                     ("bdf2", 1.0, 63, 64, "fp32"), ("theta", 1.0, 31, 128, "fp64"),
                                                     ("bdf3", 1.0, 63, 100, "fp64"), ("bdf2", 1.0, 63, 128, "fp32"),
                                                     ("theta", 0.5, 31, 256, "fp32"), ("bdf2", 1.0, 127, 200, "fp32")])
def test_tile64_single_solves(scheme, theta, N, n, pprec):
    """64-mode column tiles (single plans, ceil(n/2) <= 64): float64 equal to the oracle's
    iterate to 1e-10 at its stopping iteration; float32 within the iteration bound."""
    from paper_2201_10062_amd import Plan
    _dev()
    g = Plan(2, N, n, scheme=scheme, theta=theta, pprec=pprec, tile_cols=64)
    assert g.tile_cols == 64
    o = System(2, N, n, scheme=scheme, theta=theta)
    b = np.random.default_rng(33).standard_normal(n * g.m)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    assert info["status"] == "ok"
    if pprec == "fp64":
        assert info["iters"] == ref.iters
        assert rel(_n(x), ref.x) < 1e-10
    else:
        assert info["iters"] <= int(1.1 * ref.iters) + 1
        assert np.linalg.norm(b - o.apply_T(_n(x))) / np.linalg.norm(b) <= 1e-8


def test_tile64_rejected_beyond_hp64():
    """64-mode tiles: ceil(n/2) <= 64 in float64, <= 128 with float32 transforms."""
    from paper_2201_10062_amd import Plan, smr
    _dev()
    with pytest.raises(smr.SmrError, match="eunsupported"):
        Plan(2, 15, 160, tile_cols=64)
    assert Plan(2, 15, 160, tile_cols=64, pprec="fp32").tile_cols == 64
    with pytest.raises(smr.SmrError, match="eunsupported"):
        Plan(2, 15, 300, tile_cols=64, pprec="fp32")


def test_tile64_batched_fp32_hp128():
    """Float32 batched launches with 64-mode tiles at ceil(n/2) = 128 beside 32-mode ones
    (parity unpinned by rounding): every instance reaches the tolerance with the float64 true
    residual, within 10% (+1) of the float64 oracle's iterations."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    probs = W.bdf2_batch(count=18, Ns=(31, 63, 127), ns=(200, 256))
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, pprec="fp32", tile_cols=64 if i % 2 == 0 else 32)
             for i, p in enumerate(probs)]
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], rtol=1e-8)
    for p, x, info in zip(probs, xs, infos):
        o = System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay)
        ref = o.solve(p.b.reshape(-1), rtol=1e-8, maxit=600)
        r = np.linalg.norm(p.b.reshape(-1) - o.apply_T(_n(x))) / np.linalg.norm(p.b)
        assert info["status"] == "ok" and r <= 1e-8, (p.name, info)
        assert info["iters"] <= int(1.1 * ref.iters) + 1, (p.name, info["iters"], ref.iters)


def test_tile64_batched_classes():
    """Batched launches with 64-mode column tiles (every instance has ceil(n/2) <= 64):
    constant and variable a, BDF2 beside BDF3 (3- and 5-tap classes in separate batches), a
    class of 64-mode tiles beside a class of 32; every instance equals the oracle."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    probs = W.bdf2_batch(count=24, Ns=(15, 31, 63), ns=(16, 40, 64, 128))
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, tile_cols=64 if i % 2 == 0 else 32)
             for i, p in enumerate(probs)]
    assert {pl.tile_cols for pl in plans} - {0} == {32, 64}   # N = 15 with variable a: physical basis
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], rtol=1e-8)
    for p, x, info in zip(probs, xs, infos):
        ref = System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay).solve(p.b.reshape(-1), rtol=1e-8, maxit=600)
        assert info["status"] == "ok" and info["iters"] == ref.iters, (p.name, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-10, p.name
    # 5 time taps (BDF3) in a batch of their own, float64 and float32
    rng = np.random.default_rng(34)
    shapes = [(31, 20, "fp64"), (63, 24, "fp64"), (31, 30, "fp32")]
    plans5 = [Plan(2, N, n, scheme="bdf3", tile_cols=64, pprec=pp) for N, n, pp in shapes]
    bs = [rng.standard_normal(n * N * N) for N, n, _ in shapes]
    xs, infos = Batch(plans5).solve([_t(b) for b in bs], rtol=1e-8)
    for (N, n, pp), b, x, info in zip(shapes, bs, xs, infos):
        o = System(2, N, n, scheme="bdf3")
        ref = o.solve(b, rtol=1e-8, maxit=600)
        assert info["status"] == "ok", (N, n, pp, info)
        if pp == "fp64":
            assert info["iters"] == ref.iters and rel(_n(x), ref.x) < 1e-10, (N, n)
        else:
            assert info["iters"] <= int(1.1 * ref.iters) + 1
            assert np.linalg.norm(b - o.apply_T(_n(x))) / np.linalg.norm(b) <= 1e-8


def test_info_reports_tile_width():
    """smr_info.tile_cols: the width a solve's fused launches ran with (the plan's for single
    solves, the class's for batched ones), 0 on the physical-basis path."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    rng = np.random.default_rng(35)
    g = Plan(2, 31, 40, scheme="bdf2", tile_cols=64)
    _, info = g.solve(_t(rng.standard_normal(40 * 31 * 31)), rtol=1e-8)
    assert info["tile_cols"] == 64
    gp = Plan(2, 31, 40, scheme="bdf2", general_path=True)
    _, info = gp.solve(_t(rng.standard_normal(40 * 31 * 31)), rtol=1e-8)
    assert info["tile_cols"] == 0
    plans = [Plan(2, 31, 40, scheme="bdf2", tile_cols=16), Plan(2, 15, 40, scheme="bdf2", tile_cols=32),
             Plan(2, 31, 24, scheme="bdf2", general_path=True)]
    _, infos = Batch(plans).solve([_t(rng.standard_normal(p.n * p.m)) for p in plans], rtol=1e-8)
    assert [i["tile_cols"] for i in infos] == [16, 32, 0]
