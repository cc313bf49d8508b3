"""GPU parity: every entry point of the HIP library against the FP64 CPU oracle on the
same seeded inputs.  Operators must agree to ~1e-13 relative (max-norm), MINRES must
stop at the oracle's iteration and agree with its iterate to 1e-10 relative."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
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


def _faces(kind, N, dim, seed=0):
    if kind == "const":
        return None, None
    if kind == "var":
        rng = np.random.default_rng(seed)
        if dim == 1:
            return rng.uniform(0.5, 1.5, N + 1), None
        return rng.uniform(0.5, 1.5, (N, N + 1)), rng.uniform(0.5, 1.5, (N + 1, N))
    # smooth variable coefficient of the variable-coefficient workload
    return W.sample_faces(lambda x, y=0.0: 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * (y if dim == 2 else 0.25)), N, dim) \
        if dim == 2 else W.sample_faces(lambda x: 1.0 + 0.5 * np.sin(2 * np.pi * x), N, 1)


def _pair(dim, N, n, scheme="theta", theta=1.0, precond="PH", kind="const", cheb_k=3, general=False):
    from paper_2201_10062_amd import Plan
    ax, ay = _faces(kind, N, dim)
    g = Plan(dim, N, n, scheme=scheme, theta=theta, precond=precond, cheb_k=cheb_k, ax=ax, ay=ay,
             general_path=general)
    o = System(dim, N, n, scheme=scheme, theta=theta, ax=ax, ay=ay,
               precond={"PH": "PH", "PTHETA_CHEB": "PTHETA_CHEB", "NONE": "NONE"}[precond], cheb_k=cheb_k)
    return g, o


OPS = [
    (1, 63, 64, "theta", 1.0, "const"),
    (1, 31, 17, "theta", 0.5, "var"),
    (1, 7, 5, "bdf2", 1.0, "var"),
    (2, 31, 33, "theta", 0.5, "const"),
    (2, 63, 16, "theta", 1.0, "var"),
    (2, 127, 8, "theta", 0.3, "smooth"),
    (2, 15, 64, "bdf2", 1.0, "const"),
    (2, 31, 20, "bdf2", 1.0, "var"),
    (2, 3, 1, "theta", 1.0, "const"),
    (2, 1, 3, "theta", 0.5, "var"),
    (2, 255, 4, "theta", 1.0, "var"),
    (2, 255, 3, "bdf2", 1.0, "smooth"),
    (2, 15, 300, "bdf2", 1.0, "var"),       # hp = 256: one folded block per pass
    (2, 7, 600, "theta", 0.5, "var"),       # hp = 512
]


@pytest.mark.parametrize("dim,N,n,scheme,theta,kind", OPS)
def test_apply_A_parity(dim, N, n, scheme, theta, kind):
    g, o = _pair(dim, N, n, scheme, theta, kind=kind)
    x = np.random.default_rng(1).standard_normal(n * g.m)
    y = _n(g.apply_A(_t(x)))
    assert rel(y, o.apply_YT(x)) < 1e-13


@pytest.mark.parametrize("dim,N,n,scheme,theta,kind", OPS)
def test_apply_P_inv_parity(dim, N, n, scheme, theta, kind):
    g, o = _pair(dim, N, n, scheme, theta, kind=kind)
    v = np.random.default_rng(2).standard_normal(n * g.m)
    z = _n(g.apply_P_inv(_t(v)))
    assert rel(z, o.apply_Pinv(v)) < 1e-12


@pytest.mark.parametrize("dim,N,n,theta,k", [(2, 15, 12, 1.0, 1), (2, 31, 9, 0.5, 3), (1, 31, 16, 1.0, 4),
                                             (2, 7, 6, 1.0, 2), (2, 127, 5, 1.0, 2), (2, 255, 3, 1.0, 2),
                                             (2, 15, 300, 1.0, 2)])
def test_apply_P_theta_cheb_parity(dim, N, n, theta, k):
    g, o = _pair(dim, N, n, "theta", theta, precond="PTHETA_CHEB", kind="var", cheb_k=k)
    v = np.random.default_rng(3).standard_normal(n * g.m)
    z = _n(g.apply_P_inv(_t(v)))
    assert rel(z, o.apply_Pinv(v)) < 1e-12


def test_build_rhs_parity():
    p = W.crank_nicolson_2d_noisy(N=31, n=20)
    g, o = _pair(2, 31, 20, "theta", 0.5, kind="var")
    b = _n(g.build_rhs(_t(p.f), _t(p.u0)))
    assert rel(b, o.rhs(p.f, p.u0)) < 1e-13


MINRES_CASES = [
    (1, 63, 64, "theta", 1.0, "PH", "const"),
    (2, 31, 64, "theta", 0.5, "PH", "const"),
    (2, 31, 32, "theta", 1.0, "PH", "smooth"),
    (2, 31, 32, "bdf2", 1.0, "PH", "const"),
    (2, 15, 24, "theta", 1.0, "PTHETA_CHEB", "smooth"),
    (2, 63, 33, "theta", 0.5, "PH", "const"),
    (1, 31, 7, "bdf2", 1.0, "PH", "const"),
    (2, 7, 1, "theta", 1.0, "PH", "const"),
]


@pytest.mark.parametrize("general", [False, True], ids=["fused", "general"])
@pytest.mark.parametrize("dim,N,n,scheme,theta,precond,kind", MINRES_CASES)
def test_minres_iterate_parity(dim, N, n, scheme, theta, precond, kind, general):
    """Constant-coefficient P_H runs on the fused sine-basis kernel unless the general path
    is forced; both must reproduce the oracle's iteration count and iterate."""
    g, o = _pair(dim, N, n, scheme, theta, precond=precond, kind=kind, general=general)
    rng = np.random.default_rng(4)
    if scheme == "theta":
        f = rng.standard_normal((n + 1, g.m))
        u0 = rng.standard_normal(g.m)
        b = o.rhs(f, u0)
    else:
        b = rng.standard_normal(n * g.m)
    ref = o.solve(b, rtol=1e-8, maxit=400)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    x = _n(x)
    assert ref.status == "converged" and info["status"] == "ok"
    assert info["iters"] == ref.iters
    assert rel(x, ref.x) < 1e-10
    assert info["relres_true"] <= 1e-8
    assert abs(info["relres_true"] - ref.relres_true) <= 1e-6 * ref.relres_true + 1e-14
    assert abs(info["relres_prec"] - ref.relres_prec) <= 1e-6 * ref.relres_prec + 1e-14
    # the physical basis evaluates every true residual; the sine basis at least the initial
    # and the deciding one (the skipped ones were excluded by sqrt(min sigma) |eta|)
    if general or precond != "PH":
        assert info["res_evals"] == info["iters"] + 1
    else:
        assert 1 + (info["iters"] > 0) <= info["res_evals"] <= info["iters"] + 1


def test_minres_unpreconditioned_iterates():
    """P = I: the GPU iterate after a fixed number of steps equals the oracle's."""
    g, o = _pair(2, 15, 8, "theta", 0.5, precond="NONE")
    b = np.random.default_rng(7).standard_normal(8 * g.m)
    ref = o.solve(b, rtol=1e-300, maxit=25)
    x, info = g.solve(_t(b), rtol=1e-300, maxit=25)
    assert info["iters"] == 25 == ref.iters and info["status"] == "enotconv"
    assert rel(_n(x), ref.x) < 1e-10


def test_minres_manufactured_1d_full_size():
    """The 1D manufactured workload at its full size (N = 63, n = 64)."""
    p = W.manufactured_1d()
    g, o = _pair(1, p.N, p.n, "theta", 1.0)
    b = _n(g.build_rhs(_t(p.f), _t(p.u0)))
    ref = o.solve(o.rhs(p.f, p.u0), rtol=1e-8)
    x, info = g.solve(_t(b), rtol=1e-8)
    assert info["iters"] == ref.iters
    assert rel(_n(x), ref.x) < 1e-10


@pytest.mark.parametrize("general", [False, True], ids=["fused", "general"])
def test_minres_warm_start_and_zero_rhs_and_maxit(general):
    g, o = _pair(2, 15, 16, "theta", 0.5, general=general)
    b = np.random.default_rng(5).standard_normal(16 * g.m)
    u = o.solve_direct(b)
    x, info = g.solve(_t(b), x0=_t(u), rtol=1e-8)
    assert info["iters"] == 0 and info["status"] == "ok"
    x, info = g.solve(_t(np.zeros_like(b)), rtol=1e-8)
    assert info["iters"] == 0 and float(np.abs(_n(x)).max()) == 0.0
    for k in (1, 3):
        x, info = g.solve(_t(b), rtol=1e-14, maxit=k)
        assert info["iters"] == k and info["status"] == "enotconv"
        ref = o.solve(b, rtol=1e-300, maxit=k)
        assert rel(_n(x), ref.x) < 1e-12
    # warm start away from the solution
    x0 = 0.5 * u
    ref = o.solve(b, rtol=1e-8, x0=x0)
    x, info = g.solve(_t(b), x0=_t(x0), rtol=1e-8)
    assert info["iters"] == ref.iters and rel(_n(x), ref.x) < 1e-10


@pytest.mark.parametrize("kind,general", [("const", False), ("var", False), ("const", True)],
                         ids=["fused", "fused-var", "general"])
def test_zero_guess_equals_explicit_zero_and_in_place_guess(kind, general):
    """x0 = NULL (the initialising launch writes x = 0) gives bit for bit the iterate of an
    explicit zero guess; a guess passed in place (d_x0 == d_x) equals one passed separately."""
    import ctypes
    from paper_2201_10062_amd import smr
    g, o = _pair(2, 31, 24, "theta", 0.5, kind=kind, general=general)
    rng = np.random.default_rng(13)
    b = o.rhs(rng.standard_normal((25, g.m)), rng.standard_normal(g.m))
    bt = _t(b)
    x1, i1 = g.solve(bt, rtol=1e-9)
    x2, i2 = g.solve(bt, x0=_t(np.zeros_like(b)), rtol=1e-9)
    assert i1["iters"] == i2["iters"] and np.array_equal(_n(x1), _n(x2))
    ref = o.solve(b, rtol=1e-9)
    assert i1["iters"] == ref.iters and rel(_n(x1), ref.x) < 1e-10
    u0 = 0.3 * ref.x
    xs, is_ = g.solve(bt, x0=_t(u0), rtol=1e-9)
    xin = _t(u0)
    info = smr.SmrInfo()
    st = g.lib.smr_minres_solve(g.handle, ctypes.c_void_p(bt.data_ptr()), ctypes.c_void_p(xin.data_ptr()),
                                ctypes.c_void_p(xin.data_ptr()), 1e-9, 500, ctypes.byref(info), smr._stream())
    assert st == smr.SMR_OK and info.iters == is_["iters"]
    assert np.array_equal(_n(xin), _n(xs))
    ref0 = o.solve(b, rtol=1e-9, x0=u0)
    assert is_["iters"] == ref0.iters and rel(_n(xs), ref0.x) < 1e-10


def test_batched_initial_guesses():
    """A batch where some instances start from a guess and the others from x0 = 0 (constant
    and variable coefficients, sine-basis and physical-basis instances)."""
    from paper_2201_10062_amd import Batch, Plan
    probs = _bdf2_batch_small(12)
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay) for p in probs]
    refs0 = [System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay) for p in probs]
    x0s, want = [], []
    for i, (p, o) in enumerate(zip(probs, refs0)):
        g0 = None if i % 2 == 0 else 0.5 * o.solve_direct(p.b.reshape(-1))
        x0s.append(g0)
        want.append(o.solve(p.b.reshape(-1), rtol=1e-8, maxit=500, **({} if g0 is None else {"x0": g0})))
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], x0s=[None if g0 is None else _t(g0) for g0 in x0s],
                                   rtol=1e-8)
    for p, x, info, ref in zip(probs, xs, infos, want):
        assert info["status"] == "ok" and info["iters"] == ref.iters, (p.name, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-10, p.name


def test_adjoint_and_gradients_parity():
    N, n, theta = 15, 12, 0.5
    from paper_2201_10062_amd import Plan
    rng = np.random.default_rng(6)
    a_nodal = rng.uniform(0.7, 1.3, (N + 2, N + 2))
    g = Plan(2, N, n, theta=theta, a_nodal=a_nodal)
    o = System(2, N, n, theta=theta, a_nodal=a_nodal)
    f = rng.standard_normal((n + 1, g.m))
    u0 = rng.standard_normal(g.m)
    u = o.solve_direct(o.rhs(f, u0))
    gvec = rng.standard_normal(n * g.m)
    lam_ref = oadj.adjoint_dense(o, gvec)
    lam, info = g.solve_adjoint(_t(gvec), rtol=1e-13, maxit=400)
    assert rel(_n(lam), lam_ref) < 1e-10
    gf, gu0 = g.rhs_adjoint(_t(lam_ref))
    rf, ru0 = oadj.rhs_adjoint(o, lam_ref)
    assert rel(_n(gf), rf.reshape(-1)) < 1e-13 and rel(_n(gu0), ru0) < 1e-12
    gax, gay, gn = g.grad_a(_t(u), _t(lam_ref), u0=_t(u0))
    rx, ry = oadj.grad_faces(o, u, u0, lam_ref)
    assert rel(_n(gax), rx.reshape(-1)) < 1e-12 and rel(_n(gay), ry.reshape(-1)) < 1e-12
    assert rel(_n(gn), oadj.grad_nodal(rx, ry, N, 2).reshape(-1)) < 1e-12


@pytest.mark.parametrize("general", [False, True], ids=["fused", "general"])
def test_cn_noisy_full_size_against_direct_solve(general):
    """The 2D Crank-Nicolson workload at its full size (N = 127, n = 256): the GPU
    solution reaches the 1e-8 true residual (checked by the oracle's own matvec) and
    matches the sequential direct solve."""
    p = W.crank_nicolson_2d_noisy()
    g, o = _pair(2, p.N, p.n, "theta", 0.5, general=general)
    b = o.rhs(p.f, p.u0)
    x, info = g.solve(_t(b), rtol=1e-8)
    x = _n(x)
    assert info["status"] == "ok" and 10 <= info["iters"] <= 60
    r = np.linalg.norm(b - o.apply_T(x)) / np.linalg.norm(b)
    assert r <= 1e-8 and abs(r - info["relres_true"]) <= 1e-3 * r
    u = o.solve_direct(b)
    assert rel(x, u) < 1e-6


# ---------------------------------------------------------------- mixed precision
# Parity unpinned by design: a float32 P^{-1} is a rounding-perturbed preconditioner, so the
# iterates differ from the float64 oracle.  The checks are the ones the method fixes: the
# float64 true residual reaches the tolerance, the iteration count stays within 10% (+1) of
# the oracle's, and the solution's error against the oracle is small and reported.
@pytest.mark.parametrize("dim,N,n,scheme,theta", [(2, 31, 64, "theta", 0.5), (2, 63, 128, "theta", 1.0),
                                                  (2, 31, 64, "bdf2", 1.0), (1, 63, 64, "theta", 1.0)])
def test_mixed_fp32_solve(dim, N, n, scheme, theta):
    from paper_2201_10062_amd import Plan
    g = Plan(dim, N, n, scheme=scheme, theta=theta, pprec="fp32")
    o = System(dim, N, n, scheme=scheme, theta=theta)
    rng = np.random.default_rng(8)
    b = o.rhs(rng.standard_normal((n + 1, g.m)), rng.standard_normal(g.m)) if scheme == "theta" \
        else rng.standard_normal(n * g.m)
    ref = o.solve(b, rtol=1e-8)
    x, info = g.solve(_t(b), rtol=1e-8)
    x = _n(x)
    r = np.linalg.norm(b - o.apply_T(x)) / np.linalg.norm(b)
    err = rel(x, ref.x)
    print(f"mixed fp32 {dim}D N={N} n={n} {scheme}: iters {info['iters']} (fp64 {ref.iters}) "
          f"relres {r:.2e} err vs oracle {err:.2e}")
    assert info["status"] == "ok" and r <= 1e-8 and abs(r - info["relres_true"]) <= 1e-3 * r
    assert info["iters"] <= int(1.1 * ref.iters) + 1
    assert err < 1e-6
    # the float32 transform really ran: the iterate is not the float64 one to rounding level
    x64, _ = Plan(dim, N, n, scheme=scheme, theta=theta).solve(_t(b), rtol=1e-8)
    assert rel(x, _n(x64)) > 1e-13


@pytest.mark.parametrize("case", ["var-N15", "ptheta", "general-const", "1d-var", "hp256-var", "ptheta-N255",
                                  "ph-N255-var", "ptheta-N127", "ptheta-N63-general"])
def test_mixed_fp32_physical_basis(case):
    """Mixed precision on the physical-basis path (variable a with N + 1 outside {32, 64, 128},
    P_theta, the forced general path, 1D variable a; every spatial-transform kernel: the
    radix-2 LDS FFT, the register-FFT line tiles and the regrouped 512-point pass): float32
    time transforms and float32 intermediates of P^{-1} (each spatial pass and Chebyshev step).
    Parity unpinned by rounding; checked: the float64 true residual reaches the tolerance,
    iterations within 10% (+1) of the float64 oracle's, error vs the oracle small and reported,
    and the float32 path really ran."""
    from paper_2201_10062_amd import Plan
    dim, N, n, theta, precond, kind, general = {
        "var-N15": (2, 15, 24, 1.0, "PH", "var", False),
        "ptheta": (2, 15, 24, 1.0, "PTHETA_CHEB", "smooth", False),
        "general-const": (2, 31, 32, 0.5, "PH", "const", True),
        "1d-var": (1, 63, 64, 1.0, "PH", "var", False),
        "hp256-var": (2, 15, 300, 1.0, "PH", "var", False),
        "ptheta-N255": (2, 255, 16, 1.0, "PTHETA_CHEB", "smooth", False),
        "ph-N255-var": (2, 255, 12, 1.0, "PH", "smooth", False),
        "ptheta-N127": (2, 127, 20, 0.5, "PTHETA_CHEB", "var", False),
        "ptheta-N63-general": (2, 63, 24, 1.0, "PTHETA_CHEB", "const", True),
    }[case]
    ax, ay = _faces(kind, N, dim)
    kw = dict(scheme="theta", theta=theta, precond=precond, cheb_k=3, ax=ax, ay=ay, general_path=general)
    g = Plan(dim, N, n, pprec="fp32", **kw)
    assert g.tile_cols == 0                       # physical basis
    o = System(dim, N, n, scheme="theta", theta=theta, ax=ax, ay=ay, precond=precond, cheb_k=3)
    rng = np.random.default_rng(9)
    b = o.rhs(rng.standard_normal((n + 1, g.m)), rng.standard_normal(g.m))
    ref = o.solve(b, rtol=1e-8, maxit=400)
    x, info = g.solve(_t(b), rtol=1e-8, maxit=400)
    x = _n(x)
    r = np.linalg.norm(b - o.apply_T(x)) / np.linalg.norm(b)
    err = rel(x, ref.x)
    print(f"mixed fp32 physical basis {case}: iters {info['iters']} (fp64 {ref.iters}) relres {r:.2e} "
          f"err vs oracle {err:.2e}")
    assert info["status"] == "ok" and r <= 1e-8 and abs(r - info["relres_true"]) <= 1e-3 * r
    assert info["iters"] <= int(1.1 * ref.iters) + 1
    assert err < 1e-6
    # the float32 transform really ran: two iterations differ from the float64 ones beyond
    # rounding (converged solutions can agree far below the tolerance)
    x2, _ = g.solve(_t(b), rtol=1e-14, maxit=2, raise_on_fail=False)
    x2_64, _ = Plan(dim, N, n, **kw).solve(_t(b), rtol=1e-14, maxit=2, raise_on_fail=False)
    assert rel(_n(x2), _n(x2_64)) > 1e-11
    # smr_apply_P_inv stays float64 on a float32 plan
    v = rng.standard_normal(n * g.m)
    assert rel(_n(g.apply_P_inv(_t(v))), o.apply_Pinv(v)) < 1e-12


def test_mixed_fp32_needs_a_preconditioner():
    from paper_2201_10062_amd import Plan, SmrError
    _dev()
    with pytest.raises(SmrError):
        Plan(2, 7, 8, pprec="fp32", precond="NONE")


# ---------------------------------------------------------------- batched solves
def _bdf2_batch_small(count=12):
    """The BDF2 batch recipe at reduced sizes: N in (7, 15, 31), n in (16, 32, 64),
    a = 1 or 1 + 0.5 cos(pi x), b ~ N(0, 1)."""
    return W.bdf2_batch(count=count, Ns=(7, 15, 31), ns=(16, 32, 64))


def test_batched_matches_oracle_per_instance():
    from paper_2201_10062_amd import Batch, Plan
    probs = _bdf2_batch_small(24)
    plans = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay) for p in probs]
    xs, infos = Batch(plans).solve([_t(p.b) for p in probs], rtol=1e-8)
    for p, x, info in zip(probs, xs, infos):
        o = System(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay)
        ref = o.solve(p.b.reshape(-1), rtol=1e-8, maxit=500)
        assert info["status"] == "ok" and info["iters"] == ref.iters, (p.name, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-10, p.name


def test_batched_fp32_and_masking():
    """Constant-coefficient instances in float32 with very different iteration counts: each
    stops at its own iteration (converged instances are masked while others run)."""
    from paper_2201_10062_amd import Batch, Plan
    probs = [q for q in _bdf2_batch_small(18) if q.ax is None]
    plans = [Plan(2, p.N, p.n, scheme="bdf2", pprec="fp32") for p in probs]
    rtols = 1e-8
    bs = [_t(p.b) for p in probs]
    bs[0] = bs[0] * 0.0                       # a zero right-hand side converges at once
    xs, infos = Batch(plans).solve(bs, rtol=rtols)
    assert infos[0]["iters"] == 0 and float(_n(xs[0]).__abs__().max()) == 0.0
    for p, b, x, info in zip(probs[1:], bs[1:], xs[1:], infos[1:]):
        o = System(2, p.N, p.n, scheme="bdf2")
        ref = o.solve(p.b.reshape(-1), rtol=1e-8)
        r = np.linalg.norm(p.b.reshape(-1) - o.apply_T(_n(x))) / np.linalg.norm(p.b)
        assert info["status"] == "ok" and r <= 1e-8
        assert info["iters"] <= int(1.1 * ref.iters) + 1


def test_batched_single_and_empty():
    from paper_2201_10062_amd import Batch, Plan
    p = W.crank_nicolson_2d_noisy(N=15, n=16)
    plan = Plan(2, 15, 16, theta=0.5)
    b = plan.build_rhs(_t(p.f), _t(p.u0))
    xs, infos = Batch([plan]).solve([b], rtol=1e-8)
    x1, info1 = plan.solve(b, rtol=1e-8)
    assert infos[0]["iters"] == info1["iters"] and rel(_n(xs[0]), _n(x1)) < 1e-13
    xs, infos = Batch([]).solve([], rtol=1e-8)
    assert xs == [] and infos == []


@pytest.mark.parametrize("kind", ["const", "var"])
def test_repeated_solves_replay_captured_iterations(kind):
    """Steady iterations from the sixth on replay a graph captured at the plan's first solve.
    Several solves on one plan, with other eager work and synchronisations between them, each
    run several replays; every one must equal the oracle."""
    N, n = 31, 24
    g, o = _pair(2, N, n, "theta", 0.5, kind="var" if kind == "var" else "const")
    rng = np.random.default_rng(21)
    for rep in range(4):
        b = o.rhs(rng.standard_normal((n + 1, g.m)), rng.standard_normal(g.m))
        ref = o.solve(b, rtol=1e-11, maxit=400)
        x, info = g.solve(_t(b), rtol=1e-11, maxit=400)
        assert info["iters"] == ref.iters and info["iters"] >= 18, (rep, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-9
        y = g.apply_A(_t(b))                     # eager work between the solves
        assert rel(_n(y), o.apply_YT(b)) < 1e-12


@pytest.mark.parametrize("kind,N,n", [("const", 31, 64), ("const", 63, 40), ("var", 31, 48)],
                         ids=["const-31", "const-63", "var-31"])
def test_stop_points_and_transform_ahead(kind, N, n):
    """The host predicts the stopping iteration from the snapshots and enqueues the transform
    back from the sine basis behind the predicted last chunk, gated on the stopped state; a
    short prediction must leave it to the normal transform.  Stopping at many points (several
    tolerances, iteration limits before and inside the captured chunks), on one plan one solve
    after another, every iterate equals the oracle's at the same count."""
    g, o = _pair(2, N, n, "theta", 0.5, kind=kind)
    rng = np.random.default_rng(31)
    b = o.rhs(rng.standard_normal((n + 1, g.m)), rng.standard_normal(g.m))
    for rtol in (1e-2, 1e-4, 1e-6, 1e-7, 1e-9, 1e-11):
        ref = o.solve(b, rtol=rtol, maxit=400)
        x, info = g.solve(_t(b), rtol=rtol, maxit=400)
        assert info["status"] == "ok" and info["iters"] == ref.iters, (rtol, info, ref.iters)
        assert rel(_n(x), ref.x) < 1e-9, rtol
    for k in (2, 6, 11, 12, 17, 23):
        ref = o.solve(b, rtol=1e-300, maxit=k)
        x, info = g.solve(_t(b), rtol=1e-300, maxit=k)
        assert info["iters"] == k and info["status"] == "enotconv", (k, info)
        assert rel(_n(x), ref.x) < 1e-9, k


def test_batch_rejects_a_repeated_plan():
    """Every batch instance iterates in its own plan's vectors, so a plan may appear once."""
    from paper_2201_10062_amd import Batch, Plan, SmrError
    _dev()
    p = Plan(2, 7, 8)
    q = Plan(2, 7, 8)
    b = _t(np.ones(8 * 49))
    with pytest.raises(SmrError, match="repeated"):
        Batch([p, q, p]).solve([b, b, b])
    with pytest.raises(SmrError, match="repeated"):
        Batch([p, p]).solve_adjoint([b, b])
    xs, infos = Batch([p, q]).solve([b, b], rtol=1e-8)
    assert all(i["status"] == "ok" for i in infos)
