#!/usr/bin/env python
"""Benchmark of the MDP domain-decomposition hot path on one MI355X.

One step = one cold domain-decomposition solve of the workload (paper Sec. 3.5):
every distinct projector Q rebuilt (8M* batched AP solves each), the interface
least squares, and the reconstruction (one AP solve per subdomain).  Inputs
(boundary coefficients, geometry) are prepared before the timed region; the AP
plans (sine matrices, per-mode tridiagonal factors) persist across steps like
FFT plans.

Prints one JSON line: value = AP grid points per second over the whole step
(sum over AP solves of (n+1)(n-1), a refined solve counted once; a source adds
one AP solve per subdomain for its right-hand side), plus the per-kernel
roofline of the dominant kernel (HIP events around the dominant class's
launches in a second pass over the same number of steps; the step time comes
from the pass without events) and the CPU oracle timed on the same workload.
Workloads: uneven (default: the 16x16 layout of squares with AP grids drawn from
{128, 256, 384, 512} and k from U[20, 80], the largest single-GPU configuration),
cross_point, transmission, two_rect, bump (the cross-point layout with a source
term) and adjoint (a cold solve plus the gradient of a receiver misfit).
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

PEAKS = {  # MI355X published peaks
    "hbm": 8000.0,          # GB/s
    "f64": 78.6,            # TFLOP/s: FP64 MFMA; FP64 vector = 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
    "f32": 157.3,           # TFLOP/s (MFMA)
    "f32v": 157.3,          # TFLOP/s: FP32 vector = 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz x 2 (packed
                            # dual-issue; this build issues unpacked FP32, i.e. at most half of it)
}
ALGO = {
    # kernel class -> (bound, peak key, what "achieved" counts)
    "gemm_sine_f64": ("mfma", "f64", "flops"),
    "gemm_sine_f32": ("mfma", "f32", "flops"),
    "interface_ls": ("mfma", "f64", "flops"),
    "ap_fused_f64": ("alu", "f64", "flops"),
    "ap_fused_f32": ("alu", "f32v", "flops"),
    "chol_diag": ("alu", "f64", "flops"),
    "chol_panel": ("mfma", "f64", "flops"),
    "chol_update": ("mfma", "f64", "flops"),
    "gram": ("mfma", "f64", "flops"),
    "tridiag_f64": ("hbm", "hbm", "bytes"),
    "tridiag_f32": ("hbm", "hbm", "bytes"),
    "fold_rhs": ("hbm", "hbm", "bytes"),
    "fold_ring": ("hbm", "hbm", "bytes"),
    "residual": ("hbm", "hbm", "bytes"),
    "gather_q": ("hbm", "hbm", "bytes"),
    "unfold_grid": ("hbm", "hbm", "bytes"),
    "tridiag_adj": ("hbm", "hbm", "bytes"),
    "mf_assemble": ("hbm", "hbm", "bytes"),
    "mf_gemm": ("mfma", "f64", "flops"),
}
# kernel class -> (part of its rocprofv3 kernel name, source file) for the PMC traffic summaries
KERNELS = {
    "ap_fused_f64": ("proj_sweep_kernel<double", "paper_2103_12172_amd/csrc/proj_sweep.hip"),
    "ap_fused_f32": ("proj_sweep_kernel<float", "paper_2103_12172_amd/csrc/proj_sweep.hip"),
    "chol_diag": ("chol_diag_kernel", "paper_2103_12172_amd/csrc/ls_kernels.hip"),
    "chol_panel": ("chol_slab_kernel", "paper_2103_12172_amd/csrc/ls_kernels.hip"),
    "tridiag_f64": ("tridiag_kernel<double>", "paper_2103_12172_amd/csrc/ap_kernels.hip"),
    "gemm_sine_f64": ("gemm_bd_kernel<double", "paper_2103_12172_amd/csrc/gemm_sine.hip"),
    "gemm_sine_f32": ("gemm_bd_kernel<float", "paper_2103_12172_amd/csrc/gemm_sine.hip"),
}
COPY_BYTES = 1 << 30   # size of the calibration copy


def source_sha(path):
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy calibration), or None when there
    is none or the kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if kernel not in KERNELS or not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha(KERNELS[kernel][1]):
        return None
    return t["bytes_per_launch"]


def _counter_kib(csv_path, name_part, counter):
    """Per-dispatch values (KiB) of one counter for kernels whose name contains name_part."""
    import csv
    per = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if name_part in row["Kernel_Name"] and row["Counter_Name"] == counter:
                per[row["Dispatch_Id"]] = per.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
    return list(per.values())


def write_traffic(kernel, workload, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv):
    """profiles/traffic_<kernel>_<workload>.json from four rocprofv3 --pmc runs:
    FETCH_SIZE and WRITE_SIZE of the kernel's dispatches, and of the calibration
    copy of COPY_BYTES (bench.py --copy-calibration), which gives the scale."""
    import statistics
    name = KERNELS[kernel][0]
    fetch = _counter_kib(fetch_csv, name, "FETCH_SIZE")
    write = _counter_kib(write_csv, name, "WRITE_SIZE")
    cal_f = max(_counter_kib(cal_fetch_csv, "copyBuffer", "FETCH_SIZE"))
    cal_w = max(_counter_kib(cal_write_csv, "copyBuffer", "WRITE_SIZE"))
    sf, sw = COPY_BYTES / (cal_f * 1024.0), COPY_BYTES / (cal_w * 1024.0)
    fb = statistics.median(fetch) * 1024.0 * sf
    wb = statistics.median(write) * 1024.0 * sw
    out = {"kernel": kernel, "rocprof_name": name, "workload": workload, "dispatches": len(fetch),
           "fetch_kib_median": statistics.median(fetch), "write_kib_median": statistics.median(write),
           "copy_bytes": COPY_BYTES, "copy_fetch_kib": cal_f, "copy_write_kib": cal_w,
           "scale_fetch": sf, "scale_write": sw, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
           "bytes_per_launch": fb + wb, "source_sha": source_sha(KERNELS[kernel][1])}
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def copy_calibration(reps=3):
    """A plain device copy of COPY_BYTES (the scale of the PMC byte counters)."""
    import torch
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "reps": reps}))


def ap_points_per_step(w) -> float:
    distinct = {}
    for sd in w.subdomains:
        distinct[(sd.lx, sd.ly, sd.n, sd.k)] = sd
    pts = 0.0
    for sd in distinct.values():
        pts += 8 * w.m_star * (sd.n + 1) * (sd.n - 1)
    for sd in w.subdomains:   # reconstruction, and the source's right-hand side (step 1c) if there is one
        pts += (sd.n + 1) * (sd.n - 1) * (2 if w.source is not None else 1)
    return pts




def roofline_of(report: dict, name: str, workload: str):
    """Roofline entry of one profiled class: algorithmic work per launch over the
    class's average launch time (HIP events around each launch)."""
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
    return {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": measured_traffic(name, workload), "kernel": name,
            "avg_launch_ms": round(avg_ms, 5), "launches": r["count"],
            "algorithmic_%s_per_launch" % what: per_launch}


def roofline(report: dict, workload: str):
    # the kernel class with the most time in the step; "interface_ls" is the span of the
    # whole interface solve (its kernels are also recorded one by one), not a kernel
    name = max((k for k in report if k != "interface_ls"), key=lambda k: report[k]["total_ms"])
    return name, roofline_of(report, name, workload)


def run_steps(ctx, w, prec, sides, steps, warmup, profile, sources=None):
    """Warm-up steps (the last profiled in full to find the dominant kernel class),
    then the timed steps without instrumentation (the step time), then, when
    profiling, the same number of steps again with HIP events around the dominant
    class, the fused AP sweep and the interface span only (the rooflines; event
    records cost host time, so they stay out of the step time)."""
    import torch
    from paper_2103_12172_amd import dd, mdp
    import gc
    last = None
    selected = None
    nwarm = max(warmup, 1 if profile else 0)
    for it in range(nwarm):
        # the last warm-up step is profiled (the first one also pays one-time kernel loading)
        if profile and it == nwarm - 1:
            mdp.mdp_profile_select(ctx, None)
            mdp.mdp_profile_enable(ctx, True)
        mdp.mdp_cache_clear(ctx)
        last = dd.dd_solve(ctx, w, prec, sides=sides, want_cond=False, sources=sources)
        if profile and it == nwarm - 1:
            full = mdp.mdp_profile_report(ctx)
            mdp.mdp_profile_enable(ctx, False)
            dom = max((k for k in full if k != "interface_ls"), key=lambda k: full[k]["total_ms"])
            selected = sorted({dom, "ap_fused_f64", "interface_ls"} & (set(full) | {dom}))

    def timed():
        nonlocal last
        last = None
        gc.collect()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            mdp.mdp_cache_clear(ctx)
            last = dd.dd_solve(ctx, w, prec, sides=sides, want_cond=False, sources=sources)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    step_s = timed()
    report, prof_s = None, None
    if profile:
        mdp.mdp_profile_select(ctx, selected)
        mdp.mdp_profile_enable(ctx, True)
        prof_s = timed()
        report = mdp.mdp_profile_report(ctx)
        mdp.mdp_profile_enable(ctx, False)
        mdp.mdp_profile_select(ctx, None)
    return step_s, report, last, prof_s


def warm_ms(ctx, w, prec, sides, reps=5, sources=None):
    """DD solve with every Q already cached (the paper's convention: Q precomputed)."""
    import gc
    import torch
    from paper_2103_12172_amd import dd
    projs = dd.build_projectors(ctx, w, prec)
    dd.dd_solve(ctx, w, prec, projectors=projs, sides=sides, want_cond=False, sources=sources)
    gc.collect()                      # earlier steps' projector handles are released here, not in the timing
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        res = dd.dd_solve(ctx, w, prec, projectors=projs, sides=sides, want_cond=False, sources=sources)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        del res
    return best * 1e3




def _oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def _host_info():
    """Core count and model of the host CPU the oracle runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {"nproc": nproc, "cpu_model": model}


def _oracle_columns(sd, m_star, cols):
    """The oracle's projector columns `cols` of subdomain sd (one AP solve each); returns
    (seconds, AP grid points)."""
    import numpy as np
    from oracle.grid import APGrid
    from oracle.projector import build_projector
    from oracle.scheme import make_solver
    t0 = time.perf_counter()
    g = APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
    Q = build_projector(g, sd.k, m_star, make_solver(sd.n, g.h, sd.k), cols=np.asarray(cols))
    return time.perf_counter() - t0, float(len(cols)) * (sd.n + 1) * (sd.n - 1), Q


def _single_thread(sd, m_star, ncols):
    """The oracle restricted to one thread on ncols projector columns of sd: AP grid points/s."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        dt, pts, _ = _oracle_columns(sd, m_star, list(range(ncols)))
    return {"value": pts / dt, "unit": "AP grid-points/s", "cores": 1,
            "sample": "%d projector columns of one subdomain (n = %d), %.2f s" % (ncols, sd.n, dt)}


def cpu_baseline(w, pts, min_seconds=10.0, max_reps=3):
    """The CPU oracle, as it stands, on the same workload: full DD solves repeated
    until about min_seconds of CPU work (at most max_reps), on every core BLAS and
    LAPACK use; and on one thread, a bounded sample of projector columns."""
    from oracle import solve as osolve
    threads = _oracle_threads()
    reps, total, ores = 0, 0.0, None
    while reps < max_reps and (reps == 0 or total < min_seconds):
        t0 = time.perf_counter()
        ores = osolve.dd_solve(w)
        total += time.perf_counter() - t0
        reps += 1
    dt = total / reps
    cb = {"value": pts / dt, "unit": "AP grid-points/s", "cores": int(threads), "kind": "oracle",
          "sample": "%d full cold DD solve(s) of the same workload (every projector column by the separable "
                    "sine + LAPACK banded tridiagonal route, Householder least squares, reconstruction), "
                    "%.2f s each" % (reps, dt)}
    cb.update(_host_info())
    cb["single_thread"] = _single_thread(w.subdomains[0], w.m_star, 32)
    return ores, cb


def cpu_baseline_sampled(w, res, seed=5):
    """The CPU oracle on a bounded sample of a layout too large for a full oracle
    solve: every projector column of one seeded subdomain per distinct n (all
    cores), and a few columns of the smallest one on one thread; the sampled Q
    against the GPU's."""
    import numpy as np
    threads = _oracle_threads()
    rng = np.random.default_rng(seed)
    picks = []
    for n in sorted({sd.n for sd in w.subdomains}):
        cand = [i for i, sd in enumerate(w.subdomains) if sd.n == n]
        picks.append(int(rng.choice(cand)))
    pts, total, qerr = 0.0, 0.0, 0.0
    for i in picks:
        sd = w.subdomains[i]
        dt, p, Q = _oracle_columns(sd, w.m_star, list(range(8 * w.m_star)))
        total += dt
        pts += p
        qg = res.projectors[i].q_tensor().cpu().numpy()
        qerr = max(qerr, float(np.abs(qg - Q).max() / np.abs(Q).max()))
    cb = {"value": pts / total, "unit": "AP grid-points/s", "cores": int(threads), "kind": "oracle",
          "sample": "projectors Q of subdomains %s (n = %s, %d AP solves each by the separable sine + LAPACK "
                    "banded tridiagonal route), %.2f s in all" % (picks, [w.subdomains[i].n for i in picks],
                                                                  8 * w.m_star, total)}
    cb.update(_host_info())
    cb["single_thread"] = _single_thread(w.subdomains[picks[0]], w.m_star, 64)
    return cb, qerr


def run_adjoint(args):
    """One step = a cold DD solve of the adjoint layout (4x4 squares, n = 512, k^2 in U[400, 3600],
    64 receivers) and the gradient of J = sum |u - u_obs|^2 with respect to the 16 k^2 and every
    boundary coefficient; u_obs = the solve at k^2 (1 + 0.05 U[-1, 1]) (seeded), computed before timing."""
    import numpy as np
    import torch
    from paper_2103_12172_amd import autodiff, dd, mdp
    from paper_2103_12172_amd import workloads as wl

    w = wl.config_adjoint()
    N = len(w.subdomains)
    ctx = mdp.mdp_create(0)
    pts, own = wl.receiver_points(w, 64, 5)
    rs, rn, _ = autodiff.snap_receivers(w, pts, own)
    prob = autodiff.Problem(ctx, w, rs, rn)
    k2 = torch.tensor([sd.k ** 2 for sd in w.subdomains], dtype=torch.float64)
    _, ds = dd.side_structs(w, w.m_star)
    d = np.zeros((N, 4, w.m_star), dtype=np.complex128)
    for i in range(N):
        for s_ in range(4):
            if ds[4 * i + s_] is not None:
                d[i, s_] = ds[4 * i + s_]
    d = torch.tensor(d)
    rng = np.random.default_rng(5)
    with torch.no_grad():
        uobs = autodiff.ReceiverValues.apply(k2 * torch.tensor(1 + 0.05 * rng.uniform(-1, 1, N)), d, prob)

    def step():
        mdp.mdp_cache_clear(ctx)
        kk = k2.clone().requires_grad_(True)
        dd_ = d.clone().requires_grad_(True)
        u = autodiff.ReceiverValues.apply(kk, dd_, prob)
        J = ((u - uobs).abs() ** 2).sum()
        J.backward()
        return float(J), kk.grad, dd_.grad

    for it in range(max(args.warmup, 1)):
        if it == max(args.warmup, 1) - 1 and not args.no_profile:
            mdp.mdp_profile_select(ctx, None)
            mdp.mdp_profile_enable(ctx, True)
        step()
    report = None
    if not args.no_profile:
        report = mdp.mdp_profile_report(ctx)
        mdp.mdp_profile_enable(ctx, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        J, gk, gd = step()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    # AP solves per step: the forward (8M* columns per subdomain + its reconstruction) and the
    # gradient (per subdomain one adjoint and four forward solves)
    pts = float(sum((8 * w.m_star + 1 + 5) * (sd.n + 1) * (sd.n - 1) for sd in w.subdomains))
    line = {"metric": "AP grid-points/s (batched compact-4 Helmholtz) + DD solve ms, FP32 vs FP64",
            "value": pts / step_s, "unit": "AP grid-points/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
            "config": {"workload": w.notes + "; 64 receivers; step = cold forward solve + gradient of the misfit "
                       "with respect to 16 k^2 and all boundary coefficients", "ap_points_per_step": pts},
            "J": J, "grad_k2_max": float(gk.abs().max()), "grad_d_max": float(gd.abs().max())}
    if report:
        name, roof = roofline(report, "adjoint")
        line["roofline"] = roof
        line["kernels"] = {k: {"count": v["count"], "total_ms": round(v["total_ms"], 4)} for k, v in report.items()}
        line["kernels_note"] = "HIP-event records of the last warm-up step"
    print(json.dumps(line))
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="uneven", choices=["two_rect", "cross_point", "transmission", "bump", "uneven", "adjoint"])
    ap.add_argument("--precision", default="c128", help="c128 | c64 | c64r: precision of the reported value")
    ap.add_argument("--compare", default="c64r,c64", help="precisions also timed, comma-separated ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true", help="only run the copy that scales PMC counters")
    ap.add_argument("--write-traffic", nargs=5,
                    metavar=("KERNEL", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="reduce four rocprofv3 --pmc counter files to profiles/traffic_<kernel>_<workload>.json")
    args = ap.parse_args()

    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.workload, *args.write_traffic[1:])
        return
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
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return
    w = wl.WORKLOADS[args.workload]()
    prec = args.precision
    ctx = mdp.mdp_create(0)
    sides = dd.side_structs(w, w.m_star)
    sources = None
    if w.source is not None:
        # the source sampled on the auxiliary grids and at the foot points of gamma, resident on the
        # device before the timed region (like the boundary data)
        sources = dd.source_tensors(ctx, w, dd.build_projectors(ctx, w, prec))
        mdp.mdp_cache_clear(ctx)
    pts = ap_points_per_step(w)

    step_s, report, res, prof_s = run_steps(ctx, w, prec, sides, args.steps, args.warmup, not args.no_profile,
                                            sources)
    value = pts / step_s
    results = {prec: res}
    compare = {}
    for cp in [c for c in args.compare.split(",") if c and c != prec]:
        cstep, _, cres, _ = run_steps(ctx, w, cp, sides, max(2, args.steps // 2), 1, False, sources)
        results[cp] = cres
        compare[cp] = {"ms_per_step": round(cstep * 1e3, 4), "value": pts / cstep,
                       "dd_solve_warm_ms": round(warm_ms(ctx, w, cp, sides, sources=sources), 4)}
    warm = round(warm_ms(ctx, w, prec, sides, sources=sources), 4)

    line = {"metric": "AP grid-points/s (batched compact-4 Helmholtz) + DD solve ms, FP32 vs FP64",
            "value": value, "unit": "AP grid-points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(step_s * 1e3, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": {"c128": "c128", "c64": "c64", "c64r": "c64+f64-refine"}[prec],
            "data": "synthetic",
            "config": {"workload": w.notes, "precision": prec, "ap_points_per_step": pts,
                       "subdomains": len(w.subdomains), "m_star": w.m_star,
                       "interface_ls": "FP64 on device (semi-normal equations with refinement; %s Gram factor)"
                       % ("multifrontal" if sum(4 * w.m_star for _ in w.subdomains) > 4096 else "dense")},
            "dd_solve_cold_ms": round(step_s * 1e3, 4), "dd_solve_warm_ms": warm}
    if report:
        name, roof = roofline(report, args.workload)
        line["roofline"] = roof
        if "ap_fused_f64" in report and name != "ap_fused_f64":
            line["roofline_ap"] = roofline_of(report, "ap_fused_f64", args.workload)
        if "interface_ls" in report:
            # the interface least squares as one unit, priced at the semi-normal method's own count (Gram,
            # factor + inverse, normal solves and residuals); a Householder QR count if it fell back
            line["roofline_interface"] = roofline_of(report, "interface_ls", args.workload)
        line["kernels"] = {k: {"count": v["count"], "total_ms": round(v["total_ms"], 4)} for k, v in report.items()}
        line["kernels_note"] = ("HIP-event records of a second pass over the same number of steps (the dominant class, "
                                "the fused AP sweep and the interface span); ms_per_step comes from the pass without events")
        line["ms_per_step_profiled"] = round(prof_s * 1e3, 4)
    if compare:
        line["compare"] = compare
    if not args.no_cpu_baseline and len(w.subdomains) > 16:
        cb, qerr = cpu_baseline_sampled(w, res)
        line["cpu_baseline"] = cb
        line["error_vs_oracle"] = {prec: {"q_rel_sampled": qerr}}
    elif not args.no_cpu_baseline:
        ores, cb = cpu_baseline(w, pts)
        line["cpu_baseline"] = cb
        c_ref = np.concatenate(ores["c"])
        line["error_vs_oracle"] = {p: {"c_rel": float(np.abs(r.c.cpu().numpy() - c_ref).max() / np.abs(c_ref).max())}
                                   for p, r in results.items()}
        if w.has_exact:
            line["error_vs_exact"] = {"oracle": ores["info"]["error_max_Mplus"]}
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
