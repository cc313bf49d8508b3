"""The paper's MINRES tables (Tables 1-4 of Sec. 5: every row, tolerance 1e-6, zero initial
guess) run by the GPU solver on the paper's Examples 1 and 2 (a = 1e-5 and
a = 1e-5 sin(pi x y)), up to 16.6 M unknowns, and the errors of Table 5.

P_H column: each GPU count must equal the FP64 oracle's (golden/paper_oracle_counts.txt,
written by a script that calls only the oracle); the oracle equals the printed count on 57
of the 64 rows, and the test checks that the GPU matches the printed count on exactly those
rows.  The 7 others are Example 2 rows with m + 1 >= 128 where the paper prints 1-2 more
iterations (no reading of Kbar changes them: with a = 1e-5, tau K is negligible there).
P_theta column: against golden/paper_oracle_ptheta_counts.txt (see its test below)."""
import os

import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def _read(name):
    with open(os.path.join(HERE, "golden", name)) as fh:
        return [l.split() for l in fh if l.strip() and not l.startswith("#")]


ORACLE = {(r[0], int(r[1]), int(r[2])): (int(r[3]), int(r[4])) for r in _read("paper_oracle_counts.txt")}


@pytest.mark.parametrize("row", _read("paper_tables_full.txt"), ids=lambda r: f"{r[0]}-n{r[3]}-m{r[4]}")
def test_paper_table_iteration_count(row):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2201_10062_amd import Plan
    tab, ex, theta, n, mp1, dof, iters_ph = row[:7]
    N, n, theta = int(mp1) - 1, int(n), float(theta)
    assert n * N * N == int(dof)
    oracle_iters, paper_iters = ORACLE[(tab, n, int(mp1))]
    assert paper_iters == int(iters_ph)
    p = W.example1(N, n, theta) if ex == "1" else W.example2(N, n, theta)
    dev = torch.device("cuda:0")
    g = Plan(2, N, n, theta=theta, ax=p.ax, ay=p.ay, device=dev)
    b = g.build_rhs(torch.from_numpy(p.f.reshape(-1)).to(dev), torch.from_numpy(p.u0).to(dev))
    x, info = g.solve(b, rtol=1e-6, maxit=200)
    assert info["status"] == "ok" and info["relres_true"] <= 1e-6
    assert info["iters"] == oracle_iters, (row, info, oracle_iters)
    if oracle_iters == paper_iters:
        assert info["iters"] == paper_iters


# ---------------------------------------------------------------- Table 5 errors
@pytest.mark.parametrize("row", _read("paper_table5_full.txt"), ids=lambda r: f"n{r[0]}-m{r[1]}")
def test_paper_table5_errors(row):
    """Example 2 (exact solution e^{-t} x(1-x) y(1-y)): the GPU solutions with P_H(Kbar) and
    with P_theta (3 Chebyshev steps per mode) to the paper's tolerance 1e-6 from x0 = 0, error
    against the exact solution on the mesh.  Backward Euler: the error is the discretisation's
    and must equal the printed value (3 digits, 0.6%).  Crank-Nicolson, n <= 64: within 3.5%
    of the printed values (at n = 32 the discrete solution itself, solved directly by the
    oracle, has error 3.21e-6 where the paper prints 3.12e-6, a 3% gap from the source-term
    sampling; at n = 64 the two agree to 1%).  Crank-Nicolson, n >= 128: the printed values are
    dominated by the 1e-6 stopping error (they differ between the two preconditioners), and
    the check is only that the error stays at that scale (below 2e-6)."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import numpy as np
    from paper_2201_10062_amd import Plan
    n, mp1 = int(row[0]), int(row[1])
    N = mp1 - 1
    printed = {("BE", "PH"): float(row[3]), ("BE", "Ptheta"): float(row[4]),
               ("CN", "PH"): float(row[5]), ("CN", "Ptheta"): float(row[6])}
    dev = torch.device("cuda:0")
    exact = W.example2_exact(N, n).reshape(-1)
    errs = {}
    for scheme, theta in (("BE", 1.0), ("CN", 0.5)):
        p = W.example2(N, n, theta)
        f = torch.from_numpy(p.f.reshape(-1)).to(dev)
        u0 = torch.from_numpy(p.u0).to(dev)
        for name, kw in (("PH", {}), ("Ptheta", {"precond": "PTHETA_CHEB", "cheb_k": 3})):
            g = Plan(2, N, n, theta=theta, ax=p.ax, ay=p.ay, device=dev, **kw)
            x, info = g.solve(g.build_rhs(f, u0), rtol=1e-6, maxit=200)
            assert info["status"] == "ok" and info["relres_true"] <= 1e-6
            errs[(scheme, name)] = float(np.abs(x.cpu().numpy() - exact).max())
            del g, x
    print(f"Table 5 n={n} m+1={mp1}: " + ", ".join(f"{k[0]} {k[1]} {v:.3e} (printed {printed[k]:.3g})"
                                                   for k, v in errs.items()))
    for key, err in errs.items():
        if key[0] == "BE":
            assert abs(err - printed[key]) <= 0.006 * printed[key], key
        elif n <= 64:
            assert abs(err - printed[key]) <= 0.035 * printed[key], key
        else:
            assert err < 2e-6, key


# ---------------------------------------------------------------- P_theta columns
PTHETA = {(r[0], int(r[1]), int(r[2])): (r[3], r[4], int(r[5])) for r in _read("paper_oracle_ptheta_counts.txt")}


@pytest.mark.parametrize("row", _read("paper_tables_full.txt"), ids=lambda r: f"{r[0]}-n{r[3]}-m{r[4]}")
def test_paper_table_ptheta_count(row):
    """The P_theta column of Tables 1-4 (3 Chebyshev steps per time mode, tolerance 1e-6,
    x0 = 0): Example 1 (constant a) runs in the sine basis, where each per-mode block is
    diagonal and the solve exact; Example 2 on the physical-basis path with the Chebyshev
    per-mode solves.  Where the oracle ran the same preconditioner (golden cheb3 count, up to
    4.2 M unknowns) the GPU count equals it; beyond, Example 1 rows equal the printed count
    (the oracle equals it on every Example 1 row it ran) and Example 2 rows stop within two
    iterations below the printed one (the oracle's gap on the rows it ran)."""
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2201_10062_amd import Plan
    tab, ex, theta, n, mp1, dof = row[:6]
    N, n, theta = int(mp1) - 1, int(n), float(theta)
    exact, cheb3, printed = PTHETA[(tab, n, int(mp1))]
    assert printed == int(row[8])
    p = W.example1(N, n, theta) if ex == "1" else W.example2(N, n, theta)
    dev = torch.device("cuda:0")
    g = Plan(2, N, n, theta=theta, ax=p.ax, ay=p.ay, precond="PTHETA_CHEB", cheb_k=3, device=dev)
    assert (g.tile_cols != 0) == (ex == "1")
    b = g.build_rhs(torch.from_numpy(p.f.reshape(-1)).to(dev), torch.from_numpy(p.u0).to(dev))
    x, info = g.solve(b, rtol=1e-6, maxit=200)
    assert info["status"] == "ok" and info["relres_true"] <= 1e-6
    if cheb3 != "-":
        assert info["iters"] == int(cheb3), (row, info, cheb3)
    elif ex == "1":
        assert info["iters"] == printed, (row, info)
    else:
        assert printed - 2 <= info["iters"] <= printed, (row, info)
