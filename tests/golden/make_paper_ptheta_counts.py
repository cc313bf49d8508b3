"""Writes paper_oracle_ptheta_counts.txt: the FP64 oracle's MINRES iteration counts with the
P_theta preconditioner (def:matrix_mod_P; true relative residual <= 1e-6, zero initial
guess) for the rows of paper_tables_full.txt:
  * exact per-mode solves (sparse LU per time mode) for rows with m + 1 <= 64;
  * the fixed 3-step Chebyshev per-mode solve the library implements, for rows with at most
    4.2 M unknowns (for Example 1, a constant, it equals the exact solve).
Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_paper_ptheta_counts.py"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle.system import System  # noqa: E402

CHEB_K = 3
MAX_DOF_CHEB = 4_200_000


def main():
    rows = [l.split() for l in open(os.path.join(HERE, "paper_tables_full.txt")) if l.strip() and not l.startswith("#")]
    out = ["# FP64 oracle MINRES iterations with P_theta (def:matrix_mod_P), tolerance 1e-6 on the true",
           "# relative residual, zero initial guess, for the rows of paper_tables_full.txt.  Written by",
           "# make_paper_ptheta_counts.py.  Columns: table n m+1 exact_iters cheb3_iters paper_iters",
           "# (exact: sparse LU per time mode, m+1 <= 64; cheb3: 3-step Chebyshev per mode, DoF <= 4.2 M;",
           "# '-' where not computed)"]
    for r in rows:
        tab, ex, theta, n, mp1, dof = r[0], r[1], float(r[2]), int(r[3]), int(r[4]), int(r[5])
        N = mp1 - 1
        p = W.example1(N, n, theta) if ex == "1" else W.example2(N, n, theta)
        ex_it = ch_it = "-"
        if mp1 <= 64:
            s = System(2, N, n, theta=theta, ax=p.ax, ay=p.ay, precond="PTHETA")
            res = s.solve(s.rhs(p.f, p.u0), rtol=1e-6, maxit=200)
            assert res.status == "converged", r
            ex_it = str(res.iters)
        if dof <= MAX_DOF_CHEB:
            s = System(2, N, n, theta=theta, ax=p.ax, ay=p.ay, precond="PTHETA_CHEB", cheb_k=CHEB_K)
            res = s.solve(s.rhs(p.f, p.u0), rtol=1e-6, maxit=200)
            assert res.status == "converged", r
            ch_it = str(res.iters)
        out.append(f"{tab} {n} {mp1} {ex_it} {ch_it} {r[8]}")
        print(out[-1], flush=True)
    with open(os.path.join(HERE, "paper_oracle_ptheta_counts.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
