"""Benchmark of the fast Poisson solve on one MI355X.

Default workload: 512^3 all-Neumann vertex grid (DCT-I on every axis), second-
order finite differences, h = 1/511, right-hand side = 64 seeded Gaussian blobs
(sigma 0.02) minus its mean.  One step = one solve in FP32 with FP64 residual
refinement (fixed number of corrections) -- the forward transforms, the
eigenvalue division with the zero mode removed, the inverse transforms, the
FP64 stencil residual, zero-mode reductions and the FP64 update.  The plain
FP64 solve of the same input is timed beside it, and the CPU oracle (dense
FP64 transform matrices) is timed on the host on the same input.

Prints one JSON line (see the keys below).  Progress goes to stderr.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_solves(plan, rhs, phi, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.solve(rhs, phi)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        plan.solve(rhs, phi)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall / steps * 1e3


def kernel_roofline(records):
    """Dominant kernel (largest total time) of a profiled execute: bytes / duration."""
    by = {}
    for r in records:
        k = r["kernel"]
        e = by.setdefault(k, {"ms": 0.0, "bytes": 0.0, "count": 0})
        e["ms"] += r["ms"]
        e["bytes"] += r["bytes"]
        e["count"] += 1
    k = max(by, key=lambda x: by[x]["ms"])
    e = by[k]
    return k, e, by


def cpu_baseline(d, g):
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    axes = oracle.axes_from(d["shape"], d["h"], d["bc"], d["grid"])
    t0 = time.perf_counter()
    ref = oracle.solve(g, axes, d["approx"])
    dt = time.perf_counter() - t0
    return ref, dt, threads


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--max-iter", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver build has no multi-GPU path "
              "(the slab decomposition over RCCL is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_1409_8116_amd as mp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.n
    log(f"generating {n}^3 Neumann blob input")
    d, g = workloads.neumann_blobs(n, seed=3)
    npts = int(np.prod(d["shape"]))
    rhs = torch.tensor(g, dtype=torch.float64, device="cuda")
    phi32r = torch.empty_like(rhs)
    phi64 = torch.empty_like(rhs)

    plan_r = mp.Plan.from_desc(d, prec="f32r", max_iter=args.max_iter)
    plan_64 = mp.Plan.from_desc(d, prec="f64")
    log("timing FP32 + refinement")
    ms_r, wall_r = time_solves(plan_r, rhs, phi32r, args.steps, args.warmup)
    info_r = plan_r.info()
    log(f"  {ms_r:.3f} ms/solve, rel resid {info_r['rel_resid']:.3e}")
    log("timing FP64")
    ms_64, wall_64 = time_solves(plan_64, rhs, phi64, args.steps, args.warmup)
    info_64 = plan_64.info()
    log(f"  {ms_64:.3f} ms/solve, rel resid {info_64['rel_resid']:.3e}")

    # live per-kernel timing with HIP events on the launch stream
    prof_r = mp.Plan.from_desc(d, prec="f32r", max_iter=args.max_iter, profile=True)
    prof_64 = mp.Plan.from_desc(d, prec="f64", profile=True)
    tmp = torch.empty_like(rhs)
    recs_r, recs_64 = [], []
    for _ in range(3):
        prof_r.solve(rhs, tmp)
        recs_r += prof_r.profile()
        prof_64.solve(rhs, tmp)
        recs_64 += prof_64.profile()
    k_r, e_r, by_r = kernel_roofline(recs_r)
    k_64, e_64, _ = kernel_roofline(recs_64)
    achieved = e_r["bytes"] / (e_r["ms"] * 1e-3) / 1e9
    achieved_64 = e_64["bytes"] / (e_64["ms"] * 1e-3) / 1e9
    log(f"dominant kernel (f32r) cfg {k_r}: {e_r['count'] // 3} launches/solve, "
        f"{e_r['ms'] / e_r['count']:.3f} ms avg, {achieved:.0f} GB/s")
    log(f"dominant kernel (f64) cfg {k_64}: {e_64['ms'] / e_64['count']:.3f} ms avg, {achieved_64:.0f} GB/s")
    del prof_r, prof_64, tmp

    out = {
        "metric": "grid points solved/s (FP32+FP64 refinement to 1e-12 rel. error), with HBM GB/s",
        "value": npts / (ms_r * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_r,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"neumann_vertex_{n}^3_dct1_fd_blobs64", "shape": list(d["shape"]),
                   "bc": "N,N,N (vertex)", "approx": "fd", "refine_corrections": args.max_iter},
        "fp64_path": {"points_per_s": npts / (ms_64 * 1e-3), "ms_per_solve": ms_64,
                      "speed_ratio_f32r_over_f64": ms_64 / ms_r},
        "rel_resid": {"f32r": info_r["rel_resid"], "f64": info_64["rel_resid"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"line_pass cfg {k_r}", "launches_per_step": e_r["count"] // 3,
                     "fp64_line_pass_GBs": achieved_64},
        "wall_ms_per_step": wall_r,
    }
    if not args.no_cpu:
        log("running the CPU oracle on the same input (one full solve)")
        ref, dt, threads = cpu_baseline(d, g)
        err_r = float(torch.linalg.norm(phi32r.cpu() - torch.from_numpy(ref)) / np.linalg.norm(ref))
        err_64 = float(torch.linalg.norm(phi64.cpu() - torch.from_numpy(ref)) / np.linalg.norm(ref))
        log(f"oracle {dt:.1f} s; rel err f32r {err_r:.3e}, f64 {err_64:.3e}")
        out["cpu_baseline"] = {"value": npts / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
                               "sample": f"one full {n}^3 solve of the same input (dense FP64 transform "
                                         f"matrices, {dt:.1f} s)"}
        out["rel_err_vs_oracle"] = {"f32r": err_r, "f64": err_64}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
