#!/usr/bin/env python3
"""Benchmark of the sine-transform-preconditioned MINRES hot path on one MI355X.

Headline workload: the 64-instance BDF2 batch of uneven sizes (instance i: N = (31, 63,
127)[i % 3], n = (64, 128, 256)[(i // 3) % 3], a = 1 or 1 + 0.5 cos(pi x) when (i // 9) is
odd, b_i ~ N(0, 1) from one seed-2 stream, 66.1 M unknowns), solved to a true relative
residual of 1e-8 from x0 = 0 with Phat (Phat(Kbar) for the variable coefficient).  One step
is one solve of the whole batch in the mixed + batched form: float64 MINRES, matvec and
residual, float32 time transform and z, every iteration one per-level matvec launch per N
class and one fused launch per time-size class over all instances.  `value` is MINRES
iterations per second summed over the instances (inputs resident in HBM before the timed
region), `ms_per_step` the time-to-1e-8 of the batch; the plain float64 form (the same
plans in float64, instances one after another on one stream) is timed beside it.  The two
batched kernels are timed live with the library's HIP events on their launch stream over
the timed steps and priced against their rooflines; the FP64 CPU oracle is timed on a
bounded sample of the instances (one thread and all cores).

Extra keys: the 2D Crank-Nicolson workload (N = 127, n = 256) with its fused kernel's
roofline, the 1D manufactured solution, the largest row of each of the paper's Tables 1-4,
the N = 255, n = 512 variable-coefficient solves, and the differentiable 16-source solve.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
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

PEAK_FP64_TFLOPS = 78.6       # MI355X dense FP64 matrix peak
PEAK_FP64_VALU_TFLOPS = 78.6  # MI355X dense FP64 vector peak
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_spec_cn2d_N127_n256.json")
TRAFFIC_FILE_BATCH = os.path.join(ROOT, "profiles", "traffic_k_spec_multi_bdf2_batch64.json")
TRAFFIC_FILE_3D = os.path.join(ROOT, "profiles", "traffic_k_spec_3d_ex3_N63_n64.json")
CSRC = os.path.join(ROOT, "paper_2201_10062_amd", "csrc")


def kernel_hash(files=("k_spec.hip", "k_spec_impl.h", "mfma_tiles.h")) -> str:
    """Hash of the fused kernel's sources (its launch file, the kernel templates and the
    matrix-core tile header)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_entry(path=TRAFFIC_FILE, widths=None):
    """HBM bytes per launch of a kernel from a committed rocprofv3 --pmc summary, or None when
    the kernel's source changed since the counters were taken or when the column-tile widths
    this run launched with (`widths`: one width, or {time padding: width} per batch class)
    differ from those of the counter run (the autotuner may choose differently in another
    process, e.g. under the profiler)."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    if isinstance(widths, dict) and "per_class_bytes_per_launch" in t:
        # batches: every time-size class launches once per iteration, so the bytes per launch
        # is the mean over the classes, each at the width this run chose for it
        pc = t["per_class_bytes_per_launch"]
        if any(str(c) not in pc.get(hp, {}) for hp, c in widths.items()):
            return None
        return sum(pc[hp][str(c)] for hp, c in widths.items()) / len(widths)
    if widths is not None and t.get("tile_cols") != widths:
        return None
    return t.get("bytes_per_launch")


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count()}


def cpu_baseline_batch(probs, sample, rtol):
    """The FP64 CPU oracle timed on this host on a bounded sample of the batch's instances
    (the same seeded right-hand sides, zero initial guess, true-residual stop), once on one
    thread and once with every core (scipy.fft workers and BLAS threads = os.cpu_count();
    scipy.sparse products stay single-threaded).  Returns the baseline record and the oracle
    solutions (for the error of the GPU forms)."""
    import scipy.fft
    from threadpoolctl import threadpool_limits
    from oracle.system import System
    out = {"kind": "oracle", "unit": "iters/s", **cpu_info()}
    sols = {}
    for label, workers in (("single_thread", 1), ("all_cores", os.cpu_count() or 1)):
        with threadpool_limits(limits=workers), scipy.fft.set_workers(workers):
            t0 = time.perf_counter()
            iters = 0
            for i in sample:
                q = probs[i]
                o = System(2, q.N, q.n, scheme="bdf2", ax=q.ax, ay=q.ay)
                r = o.solve(q.b.reshape(-1), rtol=rtol, maxit=1000)
                iters += r.iters
                sols[i] = r
            dt = time.perf_counter() - t0
        out[label] = {"value": iters / dt, "iters": iters, "seconds": dt, "threads": workers}
    out["value"] = out["single_thread"]["value"]
    out["cores"] = 1
    out["sample"] = (f"instances {list(sample)} of the 64-instance BDF2 batch ({', '.join(probs[i].name for i in sample)}), "
                     f"solved to rtol {rtol} from x0 = 0; value = single-thread iters/s, all-cores beside it")
    return out, sols


def batch_algorithmic(probs, infos, pprec_bytes):
    """Algorithmic HBM bytes of the fused batched launches and bytes + flops of the per-level
    matvec launches over one batched solve, from each instance's iteration and residual counts.
    Fused launch, per degree of freedom (z in the transform precision, pprec_bytes = 4 for
    float32): init 24 + z (read b^, write v_1, z_1, x = 0), first 16 + 2 z (read z_1 or
    (T z_1)^, v_1; write v_2, z_2), steady 64 + 3 z (read z_j, z_{j-1}, v_j, v_{j-1}, w_{j-2},
    w_{j-3}, x; write v, z, w, x) less the w's that do not exist in launches 2 and 3, + 8 for
    each evaluated true residual (read b^); a variable coefficient reads (T z_j)^ (8) in place
    of z_j and evaluates its residuals in the per-level kernel.  Per-level matvec (variable a,
    launches 1 .. iters + 1): read z_j, write (T z_j)^ (z + 8), + 16 per evaluated residual
    (read x, b^); flops: four one-dimensional sine transforms per point as packed complex
    FFTs of M = 2 (N + 1) points, 2.5 M log2 M flops per line, the 5-point stencil with face
    coefficients (13 per point) and the time combination (9 per point), twice when the
    residual is evaluated."""
    import math
    z = pprec_bytes
    spec_b = ks_b = ks_f = 0.0
    for q, inf in zip(probs, infos):
        dof = q.n * q.N * q.N
        k, r = inf["iters"], inf["res_evals"]
        var = q.ax is not None
        steady = sum(64 + 3 * z + (8 - z if var else 0) - (16 if j == 2 else 8 if j == 3 else 0) for j in range(2, k + 2))
        spec_b += dof * ((24 + z) + (16 + 2 * z + (8 - z if var else 0)) + steady + (0 if var else 8 * (r - 1)))
        if var:
            M = 2 * (q.N + 1)
            per_level = 4 * q.N * 2.5 * M * math.log2(M) + 22 * q.N * q.N
            ks_b += dof * ((z + 8) * (k + 1) + 16 * (r - 1))
            ks_f += q.n * per_level * ((k + 1) + (r - 1))
    return spec_b, ks_b, ks_f


def time_padding(n: int) -> int:
    """The fused kernel's folded time rows: ceil(n/2) rounded up to 16 * 2^k."""
    hp = 16
    while hp < (n + 1) // 2:
        hp *= 2
    return hp


def batched_bdf2_headline(dev, warmup: int, steps: int, rtol: float, cpu: bool, profiled_only: bool = False,
                          matvec=None, class_widths=None):
    """The 64-instance BDF2 batch (uneven N in {31, 63, 127}, n in {64, 128, 256}, a = 1 or
    1 + 0.5 cos(pi x), b ~ N(0, 1), seed 2), inputs resident in HBM.  Mixed + batched (float64
    MINRES, matvec and residual; float32 time transform and z; every iteration one per-level
    matvec launch per N class and one fused launch per time-size class over all instances)
    is the measured form; plain float64 (the same method, instances solved back to back on one
    stream) beside it.  The kernel durations of the rooflines come from the same steps run a
    second time with the library's per-launch HIP events on (launches in sequence); with
    profiled_only only that pass runs (the command the rocprofv3 kernel trace is taken of)."""
    import torch
    import workloads as W
    from paper_2201_10062_amd import Batch, Plan, smr
    probs = W.bdf2_batch()
    bs = [torch.from_numpy(q.b.reshape(-1)).to(dev) for q in probs]
    plain = [] if profiled_only else [Plan(2, q.N, q.n, scheme="bdf2", ax=q.ax, ay=q.ay, device=dev) for q in probs]
    cw = class_widths or {}
    mixed = [Plan(2, q.N, q.n, scheme="bdf2", ax=q.ax, ay=q.ay, pprec="fp32", device=dev, matvec=matvec,
                  tile_cols=cw.get(str(time_padding(q.n)))) for q in probs]
    batch = Batch(mixed)

    def run_plain():
        return [pl.solve(b, rtol=rtol, maxit=1000) for pl, b in zip(plain, bs)]

    def run_mixed():
        xs, infos = batch.solve(bs, rtol=rtol, maxit=1000)
        return list(zip(xs, infos))

    smr.profile_enable(profiled_only)       # profiled only: every launch in sequence, warm-up included
    for _ in range(warmup):
        run_mixed()
        if not profiled_only:
            run_plain()
    torch.cuda.synchronize()
    t_mixed = float("nan")
    if not profiled_only:
        t0 = time.perf_counter()
        for _ in range(steps):
            rm = run_mixed()
        torch.cuda.synchronize()
        t_mixed = (time.perf_counter() - t0) / steps
    # kernel durations: the same steps again with the library's HIP events around every launch
    # (the launches then go one after another, without the captured graph's parallel branches)
    smr.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        rm = run_mixed()
    torch.cuda.synchronize()
    t_mixed_seq = (time.perf_counter() - t0) / steps
    smr.profile_enable(False)
    n_spec, ms_spec = smr.profile_read("spec")
    n_ks, ms_ks = smr.profile_read("kslice")
    if profiled_only:
        return {"profiled_pass_ms": t_mixed_seq * 1e3, "spec_avg_launch_us": ms_spec * 1e3 / max(n_spec, 1),
                "kslice_avg_launch_us": ms_ks * 1e3 / max(n_ks, 1)}
    t0 = time.perf_counter()
    for _ in range(steps):
        rp = run_plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    im = [i for _, i in rm]
    ip = [i for _, i in rp]
    ok = all(i["status"] == "ok" and i["relres_true"] <= rtol for i in ip + im)
    it_m, it_p = sum(i["iters"] for i in im), sum(i["iters"] for i in ip)
    ratio = max(b["iters"] / a["iters"] for a, b in zip(ip, im) if a["iters"] > 0)
    spec_b, ks_b, ks_f = batch_algorithmic(probs, im, 4)
    # the column-tile width each time-size class ran with (keyed by ceil(n/2) padded to 16 * 2^k)
    class_widths = {}
    for q, i in zip(probs, im):
        if i["tile_cols"]:
            class_widths[str(time_padding(q.n))] = i["tile_cols"]
    spec_s = ms_spec * 1e-3 / steps
    ks_s = ms_ks * 1e-3 / steps
    spec_gbs = spec_b / spec_s / 1e9
    ks_gbs = ks_b / ks_s / 1e9
    ks_tf = ks_f / ks_s / 1e12
    roof_spec = {"bound": "hbm", "achieved": spec_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                 "frac": spec_gbs / PEAK_HBM_GBS, "traffic": traffic_entry(TRAFFIC_FILE_BATCH, class_widths),
                 "class_widths": class_widths,
                 "kernel": "k_spec_multi (fused batched MINRES iteration, every time-size class)",
                 "launches": n_spec // steps, "avg_launch_us": ms_spec * 1e3 / max(n_spec, 1),
                 "bytes_per_launch": spec_b / max(n_spec // steps, 1), "kernel_ms_per_solve": ms_spec / steps}
    roof_ks = {"bound": "alu", "achieved": ks_tf, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
               "frac": ks_tf / PEAK_FP64_VALU_TFLOPS, "traffic": None,
               "kernel": "per-level U K(a) U matvec, every N class: k_kslice_multi (a level per block) or, "
                         "where timed faster, k_ks_tiles_multi (three passes over 16-line tiles, N = 127)",
               "tiled_instances": sum(pl.matvec_tiles for pl in mixed),
               "launches": n_ks // steps, "avg_launch_us": ms_ks * 1e3 / max(n_ks, 1),
               "flops_per_launch": ks_f / max(n_ks // steps, 1), "kernel_ms_per_solve": ms_ks / steps,
               "hbm_achieved_gbs": ks_gbs, "hbm_frac": ks_gbs / PEAK_HBM_GBS}
    dominant_spec = ms_spec >= ms_ks
    dof = sum(q.n * q.N * q.N for q in probs)
    rec = {
        "value": it_m / t_mixed, "ms_per_step": t_mixed * 1e3,
        "config": {"workload": "bdf2_batch64_uneven", "instances": len(probs),
                   "N": [31, 63, 127], "n": [64, 128, 256], "variable_coefficient": sum(q.ax is not None for q in probs),
                   "precond": "Phat / Phat(Kbar)", "precision": "f64 MINRES, matvec, residual; f32 time transform and z",
                   "rtol": rtol, "dof_total": dof},
        "time_to_1e-8_ms": t_mixed * 1e3, "time_to_1e-8_ms_profiled_sequential": t_mixed_seq * 1e3,
        "plain_fp64": {"time_to_1e-8_ms": t_plain * 1e3, "iters_per_s": it_p / t_plain, "iters_total": it_p},
        "speedup_mixed_batched_vs_plain": t_plain / t_mixed,
        "iters_total_mixed": it_m, "iters_total_plain": it_p, "iters_max_ratio_mixed_over_plain": ratio,
        "all_converged": ok,
        "roofline": roof_spec if dominant_spec else roof_ks,
        "roofline_other": roof_ks if dominant_spec else roof_spec,
    }
    if cpu:
        sample = (0, 1, 2, 9, 10, 11)
        base, sols = cpu_baseline_batch(probs, sample, rtol)
        rec["cpu_baseline"] = base
        errs_m, errs_p = {}, {}
        for i in sample:
            ref = sols[i].x
            sc = float(np.abs(ref).max())
            errs_m[probs[i].name] = float(np.abs(rm[i][0].cpu().numpy() - ref).max()) / sc
            errs_p[probs[i].name] = float(np.abs(rp[i][0].cpu().numpy() - ref).max()) / sc
            assert rp[i][1]["iters"] == sols[i].iters, (probs[i].name, rp[i][1]["iters"], sols[i].iters)
        rec["rel_err_vs_oracle"] = {"mixed_batched": errs_m, "plain_fp64": errs_p}
    return rec


def cn2d_leg(dev, warmup: int, steps: int, rtol: float, tile_cols=None):
    """The 2D Crank-Nicolson workload (N = 127, n = 256, a = 1, noisy source, seed 0, P_H),
    plain float64, one solve per step; the fused sine-basis iteration kernel timed with HIP
    events and priced against the HBM roofline (its two folded time GEMMs against the FP64
    matrix peak beside it); the float32-transform form beside it."""
    import torch
    import workloads as W
    from paper_2201_10062_amd import Plan, smr
    p = W.crank_nicolson_2d_noisy()          # N = 127, n = 256, theta = 1/2, seed 0
    f = torch.from_numpy(p.f.reshape(-1)).to(dev)
    u0 = torch.from_numpy(p.u0).to(dev)
    plan = Plan(2, p.N, p.n, theta=p.theta, device=dev, tile_cols=tile_cols)
    b = plan.empty()

    def step():
        plan.build_rhs(f, u0, out=b)
        return plan.solve(b, rtol=rtol)[1]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    smr.profile_enable(True)
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    smr.profile_enable(False)
    n_spec, ms_spec = smr.profile_read("spec")
    iters = [i["iters"] for i in infos]
    dof = p.n * p.m

    # Fused launch bytes per degree of freedom (float64): init 32 (read b^; write v_1, z_1,
    # x = 0), first 32 (read z_1, v_1; write v_2, z_2), steady 88 (read z_j, z_{j-1}, v_j,
    # v_{j-1}, w_{j-2}, w_{j-3}, x; write v, z, w, x) less the w's that do not exist in
    # launches 2 and 3, + 8 (read b^) for each evaluated true residual; 2 n^2 m flops of
    # folded time GEMMs per launch.
    def steady_bytes(k):
        return sum(88 - (16 if j == 2 else 8 if j == 3 else 0) for j in range(2, k + 2))
    bytes_total = sum((32 + 32 + steady_bytes(i["iters"]) + 8 * (i["res_evals"] - 1)) * dof for i in infos)
    flops_per_launch = 2.0 * p.n * p.n * p.m
    avg_launch_s = (ms_spec / n_spec) * 1e-3 if n_spec else float("nan")
    bytes_per_launch = bytes_total / max(n_spec, 1)
    achieved_gbs = bytes_per_launch / avg_launch_s / 1e9
    achieved_tf = flops_per_launch / avg_launch_s / 1e12
    out = {"workload": "cn2d_noisy_N127_n256", "dof": dof, "precond": "P_H", "pprec": "fp64", "rtol": rtol,
           "iters_per_s": sum(iters) / dt, "time_to_1e-8_ms": dt / steps * 1e3, "iters_per_solve": iters[-1],
           "residuals_evaluated_per_solve": infos[-1]["res_evals"], "relres_true": infos[-1]["relres_true"],
           "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": achieved_gbs / PEAK_HBM_GBS, "traffic": traffic_entry(widths=plan.tile_cols),
                        "tile_cols": plan.tile_cols,
                        "kernel": "k_spec (fused sine-basis MINRES iteration)", "launches": n_spec,
                        "launches_expected": sum(k + 2 for k in iters), "avg_launch_us": avg_launch_s * 1e6,
                        "bytes_per_launch": bytes_per_launch},
           "roofline_mfma": {"achieved": achieved_tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                             "frac": achieved_tf / PEAK_FP64_TFLOPS, "flops_per_launch": flops_per_launch}}
    # the same workload with the float32 preconditioner (error vs the float64 solution, which
    # equals the oracle's iterate to 1e-10 in the parity tests)
    mplan = Plan(2, p.N, p.n, theta=p.theta, pprec="fp32", device=dev)
    x64, _ = plan.solve(b, rtol=rtol)
    for _ in range(warmup):
        mplan.solve(b, rtol=rtol)
    torch.cuda.synchronize()
    tm0 = time.perf_counter()
    for _ in range(steps):
        plan.build_rhs(f, u0, out=b)
        xm, minfo = mplan.solve(b, rtol=rtol)
    torch.cuda.synchronize()
    tm1 = time.perf_counter()
    out["mixed_fp32"] = {"time_to_1e-8_ms": (tm1 - tm0) / steps * 1e3, "iters_per_solve": minfo["iters"],
                         "iters_per_s": minfo["iters"] * steps / (tm1 - tm0), "relres_true": minfo["relres_true"],
                         "rel_err_vs_fp64": float((xm - x64).abs().max() / x64.abs().max())}
    return out


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


def spec_fp64_bytes(infos, dof):
    """Algorithmic bytes of the float64 fused launches of the given solves (see cn2d_leg)."""
    def steady(k):
        return sum(88 - (16 if j == 2 else 8 if j == 3 else 0) for j in range(2, k + 2))
    return sum((32 + 32 + steady(i["iters"]) + 8 * (i["res_evals"] - 1)) * dof for i in infos)


def paper_tables_leg(dev, reps: int = 3):
    """The largest row of each of the paper's tables solved here with P_H and P_theta (3
    Chebyshev steps per mode), tolerance 1e-6, x0 = 0, beside the iteration counts and MATLAB
    CPU seconds the paper prints (dual 16-core Xeon Gold 6246R, 3.4 GHz, Sec. 5): Tables 1-4
    (2D, n = 256, m + 1 = 256, 16.6 M unknowns) and Tables 6-7 (3D Example 3, n = 64,
    m + 1 = 64, 16.0 M unknowns).  For the 3D rows the fused sine-basis kernel (with the
    grouped reduction of its partial sums) is also priced against the HBM roofline."""
    import torch
    import workloads as W
    from paper_2201_10062_amd import Plan, smr
    rows = []
    for name, dim in (("paper_tables_full.txt", 2), ("paper_tables_3d.txt", 3)):
        with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
            for line in fh:
                r = line.split()
                if not r or line.startswith("#"):
                    continue
                if dim == 2 and r[3] == "256" and r[4] == "256":
                    rows.append(dict(dim=2, table=r[0], ex=r[1], theta=float(r[2]), n=int(r[3]), mp1=int(r[4]),
                                     printed={"PH": (int(r[6]), float(r[7])), "PTHETA_CHEB": (int(r[8]), float(r[9]))}))
                if dim == 3 and r[2] == "64" and r[3] == "64":
                    rows.append(dict(dim=3, table=r[0], ex="3", theta=float(r[1]), n=int(r[2]), mp1=int(r[3]),
                                     printed={"PH": (int(r[6]), float(r[7])), "PTHETA_CHEB": (int(r[8]), float(r[9]))}))
    out = []
    for r in rows:
        N, n, theta, dim = r["mp1"] - 1, r["n"], r["theta"], r["dim"]
        p = {"1": W.example1, "2": W.example2, "3": W.example3}[r["ex"]](N, n, theta)
        dof = n * N ** dim
        f, u0 = torch.from_numpy(p.f.reshape(-1)).to(dev), torch.from_numpy(p.u0).to(dev)
        for pre in ("PH", "PTHETA_CHEB"):
            g = Plan(dim, N, n, theta=theta, ax=p.ax, ay=p.ay, az=p.az, precond=pre, cheb_k=3, device=dev)
            b = g.build_rhs(f, u0)
            g.solve(b, rtol=1e-6, maxit=200)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                x, info = g.solve(b, rtol=1e-6, maxit=200)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            e = {"table": r["table"], "dim": dim, "precond": pre, "n": n, "m_plus_1": r["mp1"], "dof": dof,
                 "path": "sine basis" if g.tile_cols else "physical basis", "iters": info["iters"],
                 "paper_iters": r["printed"][pre][0], "gpu_ms": ms, "paper_cpu_s": r["printed"][pre][1]}
            if dim == 3 and g.tile_cols:
                smr.profile_enable(True)
                _, pinfo = g.solve(b, rtol=1e-6, maxit=200)
                smr.profile_enable(False)
                nl, msl = smr.profile_read("spec")
                bpl = spec_fp64_bytes([pinfo], dof) / max(nl, 1)
                gbs = bpl / (msl / max(nl, 1) * 1e-3) / 1e9
                e["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": gbs / PEAK_HBM_GBS,
                                 "traffic": traffic_entry(TRAFFIC_FILE_3D, g.tile_cols),
                                 "kernel": "k_spec + grouped partial reduction (3D, 4D sine basis)",
                                 "launches": nl, "avg_launch_us": msl / max(nl, 1) * 1e3, "bytes_per_launch": bpl,
                                 "tile_cols": g.tile_cols}
            out.append(e)
            del g, b, x
    return out


def variable_coef_leg(dev, rtol: float, oracle: bool = True):
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
    if oracle:
        out["reduced_shape_vs_oracle"] = variable_coef_reduced_vs_oracle(dev, rtol)
    return out


def variable_coef_reduced_vs_oracle(dev, rtol: float, N: int = 63, n: int = 128):
    """The variable-coefficient recipe at a reduced shape (the oracle finishes in seconds):
    the float64 and float32-transform GPU solutions of both preconditioners against the FP64
    oracle's solution to the same tolerance (relative max-norm error), iterations beside."""
    import torch
    import workloads as W
    from oracle.system import System
    from paper_2201_10062_amd import Plan
    p = W.variable_coef_2d(N=N, n=n)
    f = torch.from_numpy(p.f.reshape(-1)).to(dev)
    u0 = torch.from_numpy(p.u0).to(dev)
    rec = {"workload": f"varcoef2d_N{N}_n{n}"}
    for name, kw in (("P_theta_cheb3", {"precond": "PTHETA_CHEB", "cheb_k": 3}), ("P_H_kbar", {"precond": "PH"})):
        o = System(2, N, n, theta=p.theta, ax=p.ax, ay=p.ay, **kw)
        ref = o.solve(o.rhs(p.f, p.u0), rtol=rtol, maxit=400)
        sc = float(np.abs(ref.x).max())
        r = {"oracle_iters": ref.iters}
        for pprec in ("fp64", "fp32"):
            g = Plan(2, N, n, theta=p.theta, ax=p.ax, ay=p.ay, device=dev, pprec=pprec, **kw)
            x, info = g.solve(g.build_rhs(f, u0), rtol=rtol, maxit=400)
            r[pprec] = {"iters": info["iters"], "rel_err_vs_oracle": float(np.abs(x.cpu().numpy() - ref.x).max()) / sc}
        rec[name] = r
    return rec


def differentiable_leg(dev, rtol: float):
    """The differentiable-solve workload (N = 127, n = 256, backward Euler, 16 Gaussian-bump
    sources, u0 = 0): loss = ||u(f, a) - u_obs||^2 at nodal a = 1 with u_obs solved at
    a = 1 + 0.3 x y; one forward (batched MINRES) + backward (batched adjoint MINRES, adjoint
    right-hand side, coefficient gradient) through torch.autograd.  The first pass at a new
    coefficient rebuilds the cached plans' tables (timed apart as setup); the timed pass reuses
    them."""
    import torch
    import workloads as W
    from paper_2201_10062_amd.autograd import clear_cache, heat_solve
    probs, a_truth = W.inverse_problem_2d()
    f = torch.from_numpy(np.stack([q.f for q in probs])).to(dev)
    clear_cache()
    with torch.no_grad():
        uobs = heat_solve(f, torch.from_numpy(a_truth).to(dev), None, rtol=rtol)

    def step():
        ft = f.clone().requires_grad_(True)
        at = torch.ones_like(torch.from_numpy(a_truth)).to(dev).requires_grad_(True)
        u = heat_solve(ft, at, None, rtol=rtol)
        loss = ((u - uobs) ** 2).sum()
        loss.backward()
        return at.grad

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()                                  # new coefficient: plan tables rebuilt in place
    torch.cuda.synchronize()
    t_first = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    ga = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    clear_cache()
    return {"workload": "inverse_problem_N127_n256_batch16", "dof_per_source": probs[0].n * probs[0].m,
            "sources": len(probs), "forward_backward_ms": ms, "first_pass_with_setup_ms": t_first,
            "setup_ms": t_first - ms, "rtol": rtol, "grad_a_norm": float(ga.norm())}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline batch (skip the Crank-Nicolson, 1D, paper-table, variable-coefficient "
                         "and differentiable legs)")
    ap.add_argument("--profiled-pass-only", action="store_true",
                    help="only the headline's profiled pass (warm-up + the timed steps with per-launch events)")
    ap.add_argument("--tile-cols", type=int, choices=[16, 32, 64], default=None,
                    help="with --only-cn2d: force the fused kernel's column-tile width (default: the set-up "
                         "timing's choice; the counter runs fix it so that they profile the width the bench "
                         "normally launches)")
    ap.add_argument("--class-widths", default=None,
                    help="with --profiled-pass-only: force the column-tile width of each time-size class, "
                         "e.g. 32:64,64:64,128:32 (time padding:width; the headline's own choice is printed in "
                         "its roofline as class_widths, and the counter runs repeat it)")
    ap.add_argument("--matvec", choices=["level", "tiles"], default=None,
                    help="with --profiled-pass-only: force the form of the N = 127 per-level matvec (default: "
                         "the one the set-up timing keeps; the counter runs profile each form this way)")
    ap.add_argument("--only-cn2d", action="store_true",
                    help="only the 2D Crank-Nicolson leg (for profiling its fused kernel)")
    ap.add_argument("--only-varcoef", action="store_true",
                    help="only the N = 255 / n = 512 variable-coefficient leg (no CPU oracle)")
    ap.add_argument("--only-tables", action="store_true",
                    help="only the paper-table leg (largest row of Tables 1-4 and 6-7, P_H and P_theta)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB three times "
                         "(the known-size kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the solver and every "
              "workload here run on a single GPU (multi-GPU sharding is design only)", file=sys.stderr)
        return 2

    import torch

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
    if args.only_cn2d:
        print(json.dumps({"cn2d": cn2d_leg(dev, args.warmup, args.steps, args.rtol, args.tile_cols)}), flush=True)
        return 0
    if args.only_varcoef:
        print(json.dumps({"variable_coefficient": variable_coef_leg(dev, args.rtol, oracle=False)}), flush=True)
        return 0
    if args.only_tables:
        print(json.dumps({"paper_tables_largest": paper_tables_leg(dev)}), flush=True)
        return 0
    if args.profiled_pass_only:
        cw = dict(kv.split(":") for kv in args.class_widths.split(",")) if args.class_widths else None
        cw = {k: int(v) for k, v in cw.items()} if cw else None
        print(json.dumps(batched_bdf2_headline(dev, args.warmup, args.steps, args.rtol, cpu=False,
                                               profiled_only=True, matvec=args.matvec, class_widths=cw)), flush=True)
        return 0
    head = batched_bdf2_headline(dev, args.warmup, args.steps, args.rtol, cpu=not args.no_cpu)
    print(f"headline done: {head['ms_per_step']:.1f} ms per batch solve", file=sys.stderr, flush=True)
    out = {
        "metric": "time-to-1e-8 residual & MINRES iters/s; mixed+batched vs plain FP64, same GPU",
        "value": head.pop("value"),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 P^-1",
        "data": "synthetic",
        "config": head.pop("config"),
        **head,
    }
    if not args.no_extras:
        out["cn2d"] = cn2d_leg(dev, args.warmup, max(args.steps, 10), args.rtol)
        out["manufactured_1d"] = manufactured_1d_leg(dev, args.rtol)
        out["paper_tables_largest"] = paper_tables_leg(dev)
        out["variable_coefficient"] = variable_coef_leg(dev, args.rtol, oracle=not args.no_cpu)
        out["differentiable"] = differentiable_leg(dev, args.rtol)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
