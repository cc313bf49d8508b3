"""Writes paper_oracle_counts_3d.txt: the FP64 oracle's MINRES iteration counts for every row
of paper_tables_3d.txt (Example 3, 3D; true relative residual <= 1e-6, zero initial guess)
with P_H and with P_theta (per-mode Chebyshev; for a constant coefficient its inner
preconditioner is exact and one step solves each mode).  Calls only the oracle and the
input generators.  Run from the repository root:
    python tests/golden/make_paper_oracle_counts_3d.py"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle.system import System  # noqa: E402


def main():
    rows = [l.split() for l in open(os.path.join(HERE, "paper_tables_3d.txt")) if l.strip() and not l.startswith("#")]
    out = ["# FP64 oracle MINRES iterations for Example 3 (3D), tolerance 1e-6 on the true relative",
           "# residual, zero initial guess, for the rows of paper_tables_3d.txt.  Written by",
           "# make_paper_oracle_counts_3d.py.  Columns: table n m+1 ph_iters ptheta_iters paper_ph paper_ptheta"]
    for r in rows:
        tab, theta, n, mp1 = r[0], float(r[1]), int(r[2]), int(r[3])
        N = mp1 - 1
        p = W.example3(N, n, theta)
        its = []
        for pre in ("PH", "PTHETA_CHEB"):
            s = System(3, N, n, theta=theta, ax=p.ax, ay=p.ay, az=p.az, precond=pre)
            res = s.solve(s.rhs(p.f, p.u0), rtol=1e-6, maxit=200)
            assert res.status == "converged", (r, pre)
            its.append(res.iters)
            del s, res
        out.append(f"{tab} {n} {mp1} {its[0]} {its[1]} {r[6]} {r[8]}")
        print(out[-1], flush=True)
    with open(os.path.join(HERE, "paper_oracle_counts_3d.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
