"""The paper's MINRES tables (Tables 1-4 of Sec. 5: every row, P_H column, tolerance 1e-6,
zero initial guess) run by the GPU solver on the paper's Examples 1 and 2 (a = 1e-5 and
a = 1e-5 sin(pi x y)), up to 16.6 M unknowns.  Each GPU count must equal the FP64 oracle's
(golden/paper_oracle_counts.txt, written by a script that calls only the oracle); the oracle
equals the printed count on 57 of the 64 rows, and the test checks that the GPU matches the
printed count on exactly those rows.  The 7 others are Example 2 rows with m + 1 >= 128
where the paper prints 1-2 more iterations (no reading of Kbar changes them: with
a = 1e-5, tau K is negligible there)."""
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
