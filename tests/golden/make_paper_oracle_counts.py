"""Writes paper_oracle_counts.txt: the FP64 oracle's MINRES iteration counts (P_H, true
relative residual <= 1e-6, zero initial guess) for every row of paper_tables_full.txt.
Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_paper_oracle_counts.py"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle.system import System  # noqa: E402


def main():
    rows = [l.split() for l in open(os.path.join(HERE, "paper_tables_full.txt")) if l.strip() and not l.startswith("#")]
    out = ["# FP64 oracle MINRES iterations (P_H; Kbar for Example 2), tolerance 1e-6 on the true",
           "# relative residual, zero initial guess, for the rows of paper_tables_full.txt.",
           "# Written by make_paper_oracle_counts.py.  Columns: table n m+1 oracle_iters paper_iters"]
    for r in rows:
        tab, ex, theta, n, mp1 = r[0], r[1], float(r[2]), int(r[3]), int(r[4])
        N = mp1 - 1
        p = W.example1(N, n, theta) if ex == "1" else W.example2(N, n, theta)
        s = System(2, N, n, theta=theta, ax=p.ax, ay=p.ay)
        res = s.solve(s.rhs(p.f, p.u0), rtol=1e-6, maxit=200)
        assert res.status == "converged", r
        out.append(f"{tab} {n} {mp1} {res.iters} {r[6]}")
        print(out[-1], flush=True)
    with open(os.path.join(HERE, "paper_oracle_counts.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
