"""GPU parity of the two forms of the N = 127 per-level matvec of the variable-coefficient
sine-basis solve (Sec. 3.1.1: each time level goes through U, the 5-point K(a) of
eqn:matrix_Km_va, and U): one workgroup per level with the level in LDS ("level"), and three
streamed passes over 16-line tiles ("tiles").  Both against the FP64 oracle's MINRES: same
iteration count, iterate to 1e-10 (the true-residual chain of the tiled form is what stops
the solve, so it is exercised too); single plans in every scheme, float32 transforms within
the iteration bound, batches mixing both forms with other N classes, the setup's timed
choice and its cache, and the full-size BDF2 shape of the batched workload."""
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
    if kind == "rand":
        rng = np.random.default_rng(seed)
        return rng.uniform(0.5, 1.5, (N, N + 1)), rng.uniform(0.5, 1.5, (N + 1, N))
    if kind == "sin":
        return W.sample_faces(lambda x, y: 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y), N, 2)
    return W.sample_faces(lambda x, y: 1.0 + 0.5 * np.cos(np.pi * x) + 0.0 * y, N, 2)


def _rhs(o, n, m, scheme, seed):
    rng = np.random.default_rng(seed)
    if scheme == "theta":
        return o.rhs(rng.standard_normal((n + 1, m)), rng.standard_normal(m))
    return rng.standard_normal(n * m)


CASES = [
    (8, "theta", 0.5, "sin"),
    (6, "theta", 1.0, "rand"),
    (5, "bdf2", 1.0, "cos"),
    (7, "bdf3", 1.0, "rand"),
    (9, "bdf4", 1.0, "sin"),
    (1, "theta", 1.0, "rand"),
]


@pytest.mark.parametrize("form", ["level", "tiles"])
@pytest.mark.parametrize("n,scheme,theta,kind", CASES)
def test_matvec_forms_match_oracle(n, scheme, theta, kind, form):
    from paper_2201_10062_amd import Plan
    _dev()
    N = 127
    ax, ay = _faces(kind, N)
    g = Plan(2, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay, matvec=form)
    assert g.tile_cols != 0 and g.matvec_tiles == (form == "tiles")
    o = System(2, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay)
    b = _rhs(o, n, g.m, scheme, 41)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    assert ref.status == "converged" and info["status"] == "ok", (info, ref.status)
    assert info["iters"] == ref.iters, (info["iters"], ref.iters)
    assert rel(_n(x), ref.x) < 1e-10
    assert abs(info["relres_true"] - ref.relres_true) <= 1e-6 * ref.relres_true + 1e-14


def test_matvec_tiles_nonzero_guess():
    """x0 given: the initialising (T x0)^ runs through the tiled source chain."""
    from paper_2201_10062_amd import Plan
    _dev()
    N, n = 127, 6
    ax, ay = _faces("rand", N)
    g = Plan(2, N, n, theta=0.5, ax=ax, ay=ay, matvec="tiles")
    o = System(2, N, n, theta=0.5, ax=ax, ay=ay)
    b = _rhs(o, n, g.m, "theta", 42)
    x0 = np.random.default_rng(43).standard_normal(n * g.m)
    ref = o.solve(b, rtol=1e-8, maxit=400, x0=x0)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400, x0=_t(x0))
    assert info["status"] == "ok" and info["iters"] == ref.iters
    assert rel(_n(x), ref.x) < 1e-10


def test_matvec_tiles_fp32():
    """Float32 transforms and z (parity unpinned by rounding): float64 true residual at the
    tolerance, iterations within 10% (+1) of the float64 oracle's, error reported."""
    from paper_2201_10062_amd import Plan
    _dev()
    N, n = 127, 16
    ax, ay = _faces("sin", N)
    o = System(2, N, n, theta=0.5, ax=ax, ay=ay)
    b = _rhs(o, n, N * N, "theta", 44)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    for form in ("level", "tiles"):
        g = Plan(2, N, n, theta=0.5, ax=ax, ay=ay, pprec="fp32", matvec=form)
        x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
        xr = _n(x)
        r = np.linalg.norm(b - o.apply_T(xr)) / np.linalg.norm(b)
        print(f"fp32 {form}: iters {info['iters']} (fp64 oracle {ref.iters}) relres {r:.2e} err {rel(xr, ref.x):.2e}")
        assert info["status"] == "ok" and r <= 1e-8
        assert info["iters"] <= int(1.1 * ref.iters) + 1
        assert rel(xr, ref.x) < 1e-6


def test_batch_mixing_matvec_forms():
    """A batch whose N = 127 instances take both forms (two matvec classes) beside N = 31 and
    63 classes and constant-coefficient instances: every instance equals the oracle."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    probs = W.bdf2_batch(count=18, Ns=(31, 63, 127), ns=(8, 12, 16))
    plans = []
    for i, p in enumerate(probs):
        form = None if p.N != 127 else ("tiles" if i % 2 == 0 else "level")
        plans.append(Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, matvec=form))
    forms = {(p.N, pl.matvec_tiles) for p, pl in zip(probs, plans) if p.ax is not None}
    assert (127, True) in forms and (127, False) in forms
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], rtol=1e-8)
    for p, x, info in zip(probs, xs, infos):
        ref = System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay).solve(p.b.reshape(-1), rtol=1e-8, maxit=600)
        assert info["status"] == "ok" and info["iters"] == ref.iters, (p.name, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-10, p.name


def test_matvec_form_tuned_and_cached():
    from paper_2201_10062_amd import Plan, smr
    _dev()
    smr.tune_reset()
    N, n = 127, 24
    ax, ay = _faces("cos", N)
    g1 = Plan(2, N, n, scheme="bdf2", ax=ax, ay=ay)
    e1, h1, m1 = smr.tune_stats()
    assert m1 >= 1
    g2 = Plan(2, N, n, scheme="bdf2", ax=ax, ay=ay)
    e2, h2, m2 = smr.tune_stats()
    assert g2.matvec_tiles == g1.matvec_tiles and m2 == m1 and h2 > h1
    print(f"N = 127, n = 24 BDF2: tiled matvec chosen: {g1.matvec_tiles}")
    # plans without the N = 127 variable-coefficient matvec report 0
    assert not Plan(2, 63, 8, scheme="bdf2", ax=_faces("cos", 63)[0], ay=_faces("cos", 63)[1]).matvec_tiles
    assert not Plan(2, 127, 8, theta=0.5).matvec_tiles


@pytest.mark.parametrize("form", ["level", "tiles"])
def test_matvec_forms_full_size_bdf2(form):
    """The batched workload's largest variable-coefficient shape (N = 127, n = 256, BDF2,
    a = 1 + 0.5 cos(pi x)) at full size: true residual 1e-8 by the oracle's matvec, and the
    oracle's sequential direct solve to 1e-6."""
    from paper_2201_10062_amd import Plan
    _dev()
    N, n = 127, 256
    ax, ay = _faces("cos", N)
    g = Plan(2, N, n, scheme="bdf2", ax=ax, ay=ay, matvec=form)
    o = System(2, N, n, scheme="bdf2", ax=ax, ay=ay)
    b = np.random.default_rng(2).standard_normal(n * g.m)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    x = _n(x)
    assert info["status"] == "ok"
    r = np.linalg.norm(b - o.apply_T(x)) / np.linalg.norm(b)
    assert r <= 1e-8 and abs(r - info["relres_true"]) <= 1e-3 * r
    assert rel(x, o.solve_direct(b)) < 1e-6


def test_batch_graph_follows_matvec_form():
    """Two batches on one workspace with the same class layout whose N = 127 instance takes
    the per-level form in one and the tiled form in the other: the second must not replay the
    first one's captured steady iterations (the fused launch reads as many matvec partials as
    its own form writes).  Both equal the oracle past the captured iterations."""
    from paper_2201_10062_amd import Batch, Plan
    _dev()
    N, n = 127, 8
    ax, ay = _faces("sin", N)
    o = System(2, N, n, scheme="bdf2", ax=ax, ay=ay)
    b = _rhs(o, n, N * N, "bdf2", 45)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    assert ref.iters > 12
    raw = None
    for form in ("level", "tiles", "level"):
        g = Plan(2, N, n, scheme="bdf2", ax=ax, ay=ay, matvec=form)
        bt = Batch([g], workspace=raw)
        raw = bt.raw_workspace
        xs, infos = bt.solve([_t(b)], rtol=1e-8, maxit=400)
        assert infos[0]["status"] == "ok" and infos[0]["iters"] == ref.iters, (form, infos[0], ref.iters)
        assert rel(_n(xs[0]), ref.x) < 1e-10, form
