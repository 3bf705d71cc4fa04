#!/usr/bin/env python
"""Benchmark of the MDP domain-decomposition hot path on one MI355X.

One step = one cold domain-decomposition solve of the workload (paper Sec. 3.5):
every distinct projector Q rebuilt (8M* batched AP solves each), the interface
least squares, and the reconstruction (one AP solve per subdomain).  Inputs
(boundary coefficients, geometry) are prepared before the timed region; the AP
plans (sine matrices, per-mode tridiagonal factors) persist across steps like
FFT plans.

Prints one JSON line: value = AP grid points per second over the whole step
(sum over AP solves of (n+1)(n-1), a refined solve counted once), plus the
per-kernel roofline of the dominant kernel (HIP events around every launch
inside the timed region) and the CPU oracle timed on the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm": 8000.0,          # GB/s
    "f64": 78.6,            # TFLOP/s (MFMA and vector)
    "f32": 157.3,           # TFLOP/s (MFMA)
}
ALGO = {
    # kernel class -> (bound, peak key, what "achieved" counts)
    "gemm_sine_f64": ("mfma", "f64", "flops"),
    "gemm_sine_f32": ("mfma", "f32", "flops"),
    "interface_ls": ("mfma", "f64", "flops"),
    "tridiag_f64": ("hbm", "hbm", "bytes"),
    "tridiag_f32": ("hbm", "hbm", "bytes"),
    "fold_rhs": ("hbm", "hbm", "bytes"),
    "residual": ("hbm", "hbm", "bytes"),
    "gather_q": ("hbm", "hbm", "bytes"),
    "unfold_grid": ("hbm", "hbm", "bytes"),
}


def ap_points_per_step(w) -> float:
    distinct = {}
    for sd in w.subdomains:
        distinct[(sd.lx, sd.ly, sd.n, sd.k)] = sd
    pts = 0.0
    for sd in distinct.values():
        pts += 8 * w.m_star * (sd.n + 1) * (sd.n - 1)
    for sd in w.subdomains:
        pts += (sd.n + 1) * (sd.n - 1)
    return pts


def roofline(report: dict):
    # the dominant single kernel class ("interface_ls" is a span of many small kernels, reported separately)
    name = max((k for k in report if k != "interface_ls"), key=lambda k: report[k]["total_ms"])
    r = report[name]
    bound, peak_key, what = ALGO.get(name, ("hbm", "hbm", "bytes"))
    avg_ms = r["total_ms"] / r["count"]
    per_launch = r[what] / r["count"]
    if what == "flops":
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        unit = "TFLOP/s"
    else:
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        unit = "GB/s"
    peak = PEAKS[peak_key]
    return name, {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                  "frac": round(achieved / peak, 4), "traffic": None, "kernel": name,
                  "avg_launch_ms": round(avg_ms, 5), "launches": r["count"]}


def run_steps(ctx, w, prec, sides, steps, warmup, profile):
    import torch
    from paper_2103_12172_amd import dd, mdp
    import gc
    last = None
    for _ in range(warmup):
        mdp.mdp_cache_clear(ctx)
        last = dd.dd_solve(ctx, w, prec, sides=sides, want_cond=False)
    last = None
    gc.collect()
    torch.cuda.synchronize()
    if profile:
        mdp.mdp_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mdp.mdp_cache_clear(ctx)
        last = dd.dd_solve(ctx, w, prec, sides=sides, want_cond=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    report = mdp.mdp_profile_report(ctx) if profile else None
    if profile:
        mdp.mdp_profile_enable(ctx, False)
    return (t1 - t0) / steps, report, last


def warm_ms(ctx, w, prec, sides, reps=5):
    """DD solve with every Q already cached (the paper's convention: Q precomputed)."""
    import gc
    import torch
    from paper_2103_12172_amd import dd
    projs = dd.build_projectors(ctx, w, prec)
    dd.dd_solve(ctx, w, prec, projectors=projs, sides=sides, want_cond=False)
    gc.collect()                      # earlier steps' projector handles are released here, not in the timing
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        res = dd.dd_solve(ctx, w, prec, projectors=projs, sides=sides, want_cond=False)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        del res
    return best * 1e3


def cpu_baseline(w, pts):
    """The CPU oracle, as it stands, on the same workload (one full DD solve)."""
    import numpy as np
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    ores = osolve.dd_solve(w)
    dt = time.perf_counter() - t0
    return ores, {"value": pts / dt, "unit": "AP grid-points/s", "cores": int(threads), "kind": "oracle",
                  "sample": "one full cold DD solve of the same workload (all projector columns by the separable "
                            "sine + LAPACK tridiagonal route, Householder least squares, reconstruction): %.2f s"
                            % dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cross_point", choices=["two_rect", "cross_point", "transmission"])
    ap.add_argument("--precision", default=None, help="c128 | c64 | c64r (default: the workload's)")
    ap.add_argument("--compare", default="c128", help="second precision timed for comparison ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2103_12172_amd import dd, mdp
    from paper_2103_12172_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = wl.WORKLOADS[args.workload]()
    prec = args.precision or w.precision
    ctx = mdp.mdp_create(0)
    sides = dd.side_structs(w, w.m_star)
    pts = ap_points_per_step(w)

    step_s, report, res = run_steps(ctx, w, prec, sides, args.steps, args.warmup, not args.no_profile)
    value = pts / step_s
    extra = {}
    if args.compare and args.compare != prec:
        cstep, creport, _ = run_steps(ctx, w, args.compare, sides, max(2, args.steps // 2), 1, False)
        extra["compare"] = {"precision": args.compare, "ms_per_step": round(cstep * 1e3, 4),
                            "value": pts / cstep, "speedup_of_%s" % prec: round(cstep / step_s, 3)}
    extra["dd_solve_warm_ms"] = round(warm_ms(ctx, w, prec, sides), 4)

    line = {"metric": "AP grid-points/s (batched compact-4 Helmholtz) + DD solve ms, FP32 vs FP64",
            "value": value, "unit": "AP grid-points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(step_s * 1e3, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": {"c128": "c128", "c64": "c64", "c64r": "c64+f64-refine"}[prec],
            "data": "synthetic",
            "config": {"workload": w.notes, "precision": prec, "ap_points_per_step": pts,
                       "subdomains": len(w.subdomains), "m_star": w.m_star,
                       "interface_ls": "FP64 Cholesky-QR2 on device"}}
    if report:
        name, roof = roofline(report)
        line["roofline"] = roof
        line["kernels"] = {k: {"count": v["count"], "total_ms": round(v["total_ms"], 4)} for k, v in report.items()}
    line.update(extra)
    if not args.no_cpu_baseline:
        ores, cb = cpu_baseline(w, pts)
        line["cpu_baseline"] = cb
        c_gpu = res.c.cpu().numpy()
        c_ref = np.concatenate(ores["c"])
        line["error_vs_oracle"] = {"c_rel": float(np.abs(c_gpu - c_ref).max() / np.abs(c_ref).max())}
        line["error_vs_exact"] = {"oracle": ores["info"]["error_max_Mplus"]}
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
