#!/usr/bin/env python3
"""Benchmark of the sine-transform-preconditioned MINRES hot path on one MI355X.

Workload (the 2D Crank-Nicolson configuration): heat equation on the unit square,
a = 1, N = 127 interior points per axis (m = 16129), n = 256 Crank-Nicolson steps,
T = 1, f from u = sin(pi x) sin(pi y) e^{-t} plus N(0, 1e-3^2) noise (seed 0),
P_H preconditioner (3D sine transform + diagonal), plain float64.

One step = assemble f_H on the GPU and run preconditioned MINRES from x0 = 0 to a true
relative residual of 1e-8.  The reported value is MINRES iterations per second over the
K timed steps (inputs resident in HBM before the timed region); time-to-1e-8 is reported
beside it.  The dominant kernel (the fused sine-basis MINRES iteration) is timed live with
HIP events on its launch stream and priced against the HBM roofline (and, beside it, its
two folded time GEMMs against the FP64 matrix peak).

Beside it: the 64-instance BDF2 batch of uneven sizes, plain float64 (instances one after
another) against mixed precision + batched (float32 time transform, one launch per size
class per iteration), time-to-1e-8 for the whole batch.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_spec_cn2d_N127_n256.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2201_10062_amd", "csrc", "k_spec.hip")
KERNEL_HDR = os.path.join(os.path.dirname(KERNEL_SRC), "mfma_tiles.h")   # its matrix-core tiles


def kernel_hash() -> str:
    """Hash of the fused kernel's sources (the kernel file and its matrix-core tile header)."""
    h = hashlib.sha256()
    for path in (KERNEL_SRC, KERNEL_HDR):
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_entry():
    """HBM bytes per launch of the time kernel from the committed rocprofv3 --pmc summary,
    or None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(p, iters: int = 40):
    """The FP64 CPU oracle timed on this host: the first `iters` MINRES iterations of
    the same workload (single thread: scipy.fft workers=1, scipy.sparse)."""
    from oracle.system import System
    s = System(2, p.N, p.n, theta=p.theta)
    fH = s.rhs(p.f, p.u0)
    t0 = time.perf_counter()
    r = s.solve(fH, rtol=1e-300, maxit=iters)
    dt = time.perf_counter() - t0
    return {"value": r.iters / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"first {r.iters} MINRES iterations of the N=127, n=256 Crank-Nicolson workload "
                      f"(P_H, true residual each iteration), {dt:.1f} s on one host core"}


def batched_bdf2_leg(dev, warmup: int, steps: int, rtol: float):
    """The 64-instance BDF2 batch (uneven N in {31, 63, 127}, n in {64, 128, 256}, a = 1 or
    1 + 0.5 cos(pi x), b ~ N(0, 1), seed 2): plain float64 (the same method, instances solved
    back to back on one stream) against mixed + batched (float32 time transform, every
    iteration one launch per size class over all instances).  Inputs resident in HBM."""
    import torch
    import workloads as W
    from paper_2201_10062_amd import Batch, Plan
    probs = W.bdf2_batch()
    bs = [torch.from_numpy(p.b.reshape(-1)).to(dev) for p in probs]
    plain = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, device=dev) for p in probs]
    mixed = [Plan(2, p.N, p.n, scheme="bdf2", ax=p.ax, ay=p.ay, pprec="fp32", device=dev) for p in probs]
    batch = Batch(mixed)

    def run_plain():
        return [pl.solve(b, rtol=rtol, maxit=1000)[1] for pl, b in zip(plain, bs)]

    def run_mixed():
        return batch.solve(bs, rtol=rtol, maxit=1000)[1]

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            infos = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, infos

    t_plain, ip = timed(run_plain)
    t_mixed, im = timed(run_mixed)
    ok = all(i["status"] == "ok" and i["relres_true"] <= rtol for i in ip + im)
    it_p = [i["iters"] for i in ip]
    it_m = [i["iters"] for i in im]
    ratio = max(b / a for a, b in zip(it_p, it_m) if a > 0)
    nvar = sum(p.ax is not None for p in probs)
    dof = sum(p.n * p.N * p.N for p in probs)
    return {"workload": "bdf2_batch64_uneven", "instances": len(probs), "variable_coefficient": nvar,
            "dof_total": dof, "rtol": rtol,
            "plain_fp64_sequential_ms": t_plain * 1e3, "mixed_fp32_batched_ms": t_mixed * 1e3,
            "speedup": t_plain / t_mixed,
            "iters_total_plain": sum(it_p), "iters_total_mixed": sum(it_m),
            "iters_max_ratio_mixed_over_plain": ratio, "all_converged": ok,
            "mixed_iters_per_s": sum(it_m) / t_mixed, "plain_iters_per_s": sum(it_p) / t_plain}


def manufactured_1d_leg(dev, rtol: float, reps: int = 20):
    """The 1D manufactured-solution workload (N = 63, n = 64, backward Euler, a = 1,
    u = sin(pi x) e^t, 4032 unknowns): latency-bound, so time-to-tolerance per solve, the
    launches it takes, and the max error against the exact solution."""
    import math
    import torch
    import workloads as W
    from paper_2201_10062_amd import Plan
    p = W.manufactured_1d()
    g = Plan(1, p.N, p.n, theta=p.theta, device=dev)
    f = torch.from_numpy(p.f.reshape(-1)).to(dev)
    u0 = torch.from_numpy(p.u0).to(dev)
    b = g.build_rhs(f, u0)
    g.solve(b, rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.build_rhs(f, u0, out=b)
        x, info = g.solve(b, rtol=rtol)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    xs = (np.arange(1, p.N + 1) / (p.N + 1))
    t = np.arange(1, p.n + 1) / p.n
    exact = np.sin(math.pi * xs)[None, :] * np.exp(t)[:, None]
    err = float(np.abs(x.cpu().numpy().reshape(p.n, p.N) - exact).max())
    return {"workload": "manufactured1d_N63_n64", "dof": p.n * p.N, "time_to_tol_ms": ms,
            "iters": info["iters"], "rtol": rtol, "max_err_vs_exact": err}


def paper_tables_leg(dev, reps: int = 3):
    """The largest row of each of the paper's Tables 1-4 (n = 256, m + 1 = 256, 16.6 M
    unknowns, tolerance 1e-6, P_H) solved here, beside the iteration counts and MATLAB CPU
    seconds the paper prints for them (dual 16-core Xeon Gold 6246R, 3.4 GHz, Sec. 5)."""
    import torch
    import workloads as W
    from paper_2201_10062_amd import Plan
    rows = []
    path = os.path.join(ROOT, "tests", "golden", "paper_tables_full.txt")
    with open(path) as fh:
        for line in fh:
            r = line.split()
            if r and not line.startswith("#") and r[3] == "256" and r[4] == "256":
                rows.append(r)
    out = []
    for r in rows:
        tab, ex, theta, n, mp1 = r[0], r[1], float(r[2]), int(r[3]), int(r[4])
        N = mp1 - 1
        p = W.example1(N, n, theta) if ex == "1" else W.example2(N, n, theta)
        g = Plan(2, N, n, theta=theta, ax=p.ax, ay=p.ay, device=dev)
        b = g.build_rhs(torch.from_numpy(p.f.reshape(-1)).to(dev), torch.from_numpy(p.u0).to(dev))
        g.solve(b, rtol=1e-6, maxit=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x, info = g.solve(b, rtol=1e-6, maxit=200)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        out.append({"table": tab, "n": n, "m_plus_1": mp1, "dof": n * N * N, "iters": info["iters"],
                    "paper_iters": int(r[6]), "gpu_ms": ms, "paper_cpu_s": float(r[7])})
        del g, b, x
    return out


def variable_coef_leg(dev, rtol: float):
    """The variable-coefficient workload (N = 255, n = 512, backward Euler,
    a = 1 + 0.5 sin(2 pi x) sin(2 pi y) at faces, f ~ U(-1, 1), seed 1): P_theta with the
    3-step Chebyshev per-mode solve, and P_H(Kbar) beside it, each in float64 and with the
    time transforms on the float32 matrix cores (physical-basis path); the mixed-precision
    results carry their error against the float64 GPU solution."""
    import torch
    import workloads as W
    from paper_2201_10062_amd import Plan
    p = W.variable_coef_2d()
    f = torch.from_numpy(p.f.reshape(-1)).to(dev)
    u0 = torch.from_numpy(p.u0).to(dev)
    out = {"workload": f"varcoef2d_N{p.N}_n{p.n}", "dof": p.n * p.m, "rtol": rtol}
    for name, kw in (("P_theta_cheb3", {"precond": "PTHETA_CHEB", "cheb_k": 3}), ("P_H_kbar", {})):
        x64 = None
        for pprec in ("fp64", "fp32"):
            g = Plan(2, p.N, p.n, theta=p.theta, ax=p.ax, ay=p.ay, device=dev, pprec=pprec, **kw)
            b = g.build_rhs(f, u0)
            g.solve(b, rtol=rtol, maxit=400)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = g.solve(b, rtol=rtol, maxit=400)
            torch.cuda.synchronize()
            rec = {"time_to_tol_ms": (time.perf_counter() - t0) * 1e3, "iters": info["iters"],
                   "relres_true": info["relres_true"], "status": info["status"]}
            if pprec == "fp64":
                x64 = x
                out[name] = rec
            else:
                rec["rel_err_vs_fp64"] = float((x - x64).abs().max() / x64.abs().max())
                out[name]["mixed_fp32"] = rec
            del g, b
        del x, x64
    return out


def differentiable_leg(dev, rtol: float):
    """The differentiable-solve workload (N = 127, n = 256, backward Euler, 16 Gaussian-bump
    sources, u0 = 0): loss = ||u(f, a) - u_obs||^2 at nodal a = 1 with u_obs solved at
    a = 1 + 0.3 x y; one forward (batched MINRES) + backward (batched adjoint MINRES, adjoint
    right-hand side, coefficient gradient) through torch.autograd."""
    import torch
    import workloads as W
    from paper_2201_10062_amd.autograd import heat_solve
    probs, a_truth = W.inverse_problem_2d()
    f = torch.from_numpy(np.stack([q.f for q in probs])).to(dev)
    with torch.no_grad():
        uobs = heat_solve(f, torch.from_numpy(a_truth).to(dev), None, rtol=rtol)

    def step():
        ft = f.clone().requires_grad_(True)
        at = torch.ones_like(torch.from_numpy(a_truth)).to(dev).requires_grad_(True)
        u = heat_solve(ft, at, None, rtol=rtol)
        loss = ((u - uobs) ** 2).sum()
        loss.backward()
        return at.grad

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ga = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    return {"workload": "inverse_problem_N127_n256_batch16", "dof_per_source": probs[0].n * probs[0].m,
            "sources": len(probs), "forward_backward_ms": ms, "rtol": rtol,
            "grad_a_norm": float(ga.norm())}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true",
                    help="only the headline workload (skip the batch, paper-table, variable-coefficient "
                         "and differentiable legs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB three times "
                         "(the known-size kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solve runs on one GPU)", file=sys.stderr)
        return 2

    import torch
    import workloads as W
    from paper_2201_10062_amd import Plan, smr

    dev = torch.device("cuda:0")
    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.full((nel,), 1.0, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration_mib,
                          "bytes_read": nel * 8, "bytes_written": nel * 8}), flush=True)
        return 0
    p = W.crank_nicolson_2d_noisy()          # N = 127, n = 256, theta = 1/2, seed 0
    f = torch.from_numpy(p.f.reshape(-1)).to(dev)
    u0 = torch.from_numpy(p.u0).to(dev)
    plan = Plan(2, p.N, p.n, theta=p.theta, device=dev)
    b = plan.empty()

    def step():
        plan.build_rhs(f, u0, out=b)
        x, info = plan.solve(b, rtol=args.rtol)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    smr.profile_enable(True)
    iters = []
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = step()
        iters.append(info["iters"])
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    smr.profile_enable(False)
    n_spec, ms_spec = smr.profile_read("spec")
    dt = t1 - t0
    total_iters = sum(iters)
    dof = p.n * p.m
    # Dominant kernel: the fused sine-basis MINRES iteration (one launch per iteration,
    # plus one initialising launch per solve).  Algorithmic HBM bytes per degree of freedom:
    #   init 32 (zero guess: read b^; write v_1, z_1, x = 0), first 32 (read z_1, v_1; write
    #   v_2, z_2), steady 88 (read z_j, z_{j-1}, v_j, v_{j-1}, w_{j-2}, w_{j-3}, x; write v, z,
    #   w, x), less the w's that do not exist yet in launches 2 (w_0, w_-1) and 3 (w_0),
    #   plus 8 (read b^) in the launches that evaluate the true residual (the library reports
    #   how many it evaluated, the initial one included).
    # Each launch also does the two folded time GEMMs: 2 n^2 m flops.
    def steady_bytes(k):
        return sum(88 - (16 if j == 2 else 8 if j == 3 else 0) for j in range(2, k + 2))
    bytes_total = sum((32 + 32 + steady_bytes(i["iters"]) + 8 * (i["res_evals"] - 1)) * dof for i in infos)
    launches_expected = sum(k + 2 for k in iters)
    flops_per_launch = 2.0 * p.n * p.n * p.m
    avg_launch_s = (ms_spec / n_spec) * 1e-3 if n_spec else float("nan")
    bytes_per_launch = bytes_total / max(n_spec, 1)
    achieved_gbs = bytes_per_launch / avg_launch_s / 1e9
    achieved_tf = flops_per_launch / avg_launch_s / 1e12
    traffic = traffic_entry()
    out = {
        "metric": "MINRES iters/s to 1e-8 true relative residual (time-to-1e-8 beside it)",
        "value": total_iters / dt,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cn2d_noisy_N127_n256", "dim": 2, "N": p.N, "n": p.n, "m": p.m,
                   "theta": p.theta, "precond": "P_H", "pprec": "fp64", "rtol": args.rtol, "dof": dof},
        "iters_per_solve": iters[-1],
        "residuals_evaluated_per_solve": infos[-1]["res_evals"],
        "time_to_1e-8_ms": dt / args.steps * 1e3,
        "relres_true": infos[-1]["relres_true"],
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_spec (fused sine-basis MINRES iteration)",
                     "launches": n_spec, "launches_expected": launches_expected,
                     "avg_launch_us": avg_launch_s * 1e6, "bytes_per_launch": bytes_per_launch},
        "roofline_mfma": {"achieved": achieved_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                          "frac": achieved_tf / PEAK_FP64_TFLOPS, "flops_per_launch": flops_per_launch},
    }
    # the same workload with the float32 preconditioner (error vs the float64 solution reported)
    mplan = Plan(2, p.N, p.n, theta=p.theta, pprec="fp32", device=dev)
    x64, _ = plan.solve(b, rtol=args.rtol)
    for _ in range(args.warmup):
        mplan.solve(b, rtol=args.rtol)
    torch.cuda.synchronize()
    tm0 = time.perf_counter()
    for _ in range(args.steps):
        plan.build_rhs(f, u0, out=b)
        xm, minfo = mplan.solve(b, rtol=args.rtol)
    torch.cuda.synchronize()
    tm1 = time.perf_counter()
    out["mixed_fp32"] = {"time_to_1e-8_ms": (tm1 - tm0) / args.steps * 1e3, "iters_per_solve": minfo["iters"],
                         "iters_per_s": minfo["iters"] * args.steps / (tm1 - tm0),
                         "relres_true": minfo["relres_true"],
                         "rel_err_vs_fp64": float((xm - x64).abs().max() / x64.abs().max())}
    if not args.no_batch:
        out["batched_bdf2"] = batched_bdf2_leg(dev, warmup=1, steps=2, rtol=args.rtol)
        out["manufactured_1d"] = manufactured_1d_leg(dev, args.rtol)
        out["paper_tables_largest"] = paper_tables_leg(dev)
        out["variable_coefficient"] = variable_coef_leg(dev, args.rtol)
        out["differentiable"] = differentiable_leg(dev, args.rtol)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
