"""Benchmark of the fast Poisson solve on one MI355X.

Headline (one JSON line on stdout): the 512^3 all-Neumann vertex grid (DCT-I
on every axis), second-order finite differences, h = 1/511, right-hand side =
64 seeded Gaussian blobs (sigma 0.02) minus their trapezoid-weighted mean.
One step = one solve in FP32 with FP64 residual refinement (fixed number of
corrections): forward transforms, eigenvalue division with the zero mode
removed, inverse transforms, FP64 stencil residual, zero-mode reductions and
FP64 update.  The plain FP64 solve of the same input is timed beside it, and
the CPU oracle (dense FP64 transform matrices) on the host.

The same line carries the other workloads under "configs" (default
`--workload all`; `--workload NAME` prints that one alone):
  periodic32  32^3 periodic FD, FP64: us per solve, eager and graph-replayed
  mixed256    256^3 staggered P/D/N box, FP64 and FP32, FD and pseudo-spectral
  batch2048   2048 independent 2D grids (sides 64..1024), FP32 + refinement,
              autotuned plans
  channel     1024x512x256 channel, graph-captured FP32 + refinement, a stream
              of right-hand sides
  projection  one projection step (divergence, solve, velocity and pressure
              correction) on the staggered 1024x512x256 channel, FP64 fused
              and FP32 + refinement
  copy        plain 1 GiB device-to-device copy (calibrates the HBM byte counters)
Each entry: ms per step, grid points/s, algorithmic HBM GB/s and the error
against the oracle on its sample.  Progress goes to stderr.
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


def timed(fn, steps, warmup):
    """Average ms per call of fn() over `steps` calls after `warmup`, by HIP events."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall / steps * 1e3


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("line_pass.h", "cfgs.h", "specs.h"):
        with open(os.path.join(ROOT, "paper_1409_8116_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter profile, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "line_pass_neumann512_hbm_counters.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    want = kernel_sources_hash()
    for ln in lines:
        if ln.startswith("traffic:"):
            kv = dict(x.split("=", 1) for x in ln[len("traffic:"):].strip().split(" ") if "=" in x)
            if kv.get("sources") == want and kv.get("kernel", "").replace(" ", "") == kernel.replace(" ", ""):
                return float(kv["bytes_per_launch"])
    return None


def kernel_name(k):
    if k == 100:
        return "resid_kernel"
    if k == 101:
        return "finalize_kernel"
    import paper_1409_8116_amd as mp
    return mp.kernel_shape_name(k)


def kernel_roofline(records, reps):
    """Dominant kernel (largest total time) of profiled executes: algorithmic
    bytes of its launches / their HIP-event durations."""
    by = {}
    for r in records:
        e = by.setdefault(r["kernel"], {"ms": 0.0, "bytes": 0.0, "count": 0})
        e["ms"] += r["ms"]
        e["bytes"] += r["bytes"]
        e["count"] += 1
    k = max(by, key=lambda x: by[x]["ms"])
    e = by[k]
    achieved = e["bytes"] / (e["ms"] * 1e-3) / 1e9
    name = kernel_name(k)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name), "kernel": name,
            "launches_per_step": e["count"] // reps, "avg_launch_ms": e["ms"] / e["count"],
            "bytes_per_launch": e["bytes"] / e["count"]}


def profile_plan(make_plan, rhs, reps=3):
    """Per-launch HIP-event records of `reps` executes of a profiling plan."""
    import torch
    plan = make_plan()
    tmp = torch.empty_like(rhs)
    recs = []
    for _ in range(reps):
        plan.solve(rhs, tmp)
        recs += plan.profile()
    plan.close()
    return recs, reps


def step_gbs(records, reps, ms):
    """Algorithmic bytes of one step (all launches) / its time."""
    return sum(r["bytes"] for r in records) / reps / (ms * 1e-3) / 1e9


def cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count()


def cpu_oracle(d, g):
    import oracle
    axes = oracle.axes_from(d["shape"], d["h"], d["bc"], d["grid"])
    t0 = time.perf_counter()
    ref = oracle.solve(g, axes, d["approx"])
    return ref, time.perf_counter() - t0, cpu_threads()


def rel(a, ref):
    import torch
    return float(torch.linalg.norm(a.double().cpu() - torch.from_numpy(ref)) / np.linalg.norm(ref))


def base_record(args, metric, value, unit, ms, dtype, config):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# ----------------------------------------------------------------------------- workloads
def run_neumann(args):
    import torch
    import workloads
    import paper_1409_8116_amd as mp
    n = args.n
    log(f"[neumann512] generating {n}^3 Neumann blob input")
    d, g = workloads.neumann_blobs(n, seed=3)
    npts = int(np.prod(d["shape"]))
    rhs = torch.tensor(g, dtype=torch.float64, device="cuda")
    phi_r = torch.empty_like(rhs)
    phi_64 = torch.empty_like(rhs)
    plan_r = mp.Plan.from_desc(d, prec="f32r", max_iter=args.max_iter, f64_arith=args.f64_arith)
    plan_64 = mp.Plan.from_desc(d, prec="f64")
    log("[neumann512] timing FP32 + refinement")
    ms_r, wall_r = timed(lambda: plan_r.solve(rhs, phi_r), args.steps, args.warmup)
    info_r = plan_r.info()
    log(f"[neumann512]   {ms_r:.3f} ms/solve, rel resid {info_r['rel_resid']:.3e}")
    log("[neumann512] timing FP64")
    ms_64, _ = timed(lambda: plan_64.solve(rhs, phi_64), args.steps, args.warmup)
    info_64 = plan_64.info()
    log(f"[neumann512]   {ms_64:.3f} ms/solve, rel resid {info_64['rel_resid']:.3e}")
    rec_r, reps = profile_plan(lambda: mp.Plan.from_desc(d, prec="f32r", max_iter=args.max_iter, profile=True,
                                                         f64_arith=args.f64_arith), rhs)
    rec_64, _ = profile_plan(lambda: mp.Plan.from_desc(d, prec="f64", profile=True), rhs)
    roof, roof64 = kernel_roofline(rec_r, reps), kernel_roofline(rec_64, reps)
    log(f"[neumann512] dominant kernel (f32r) {roof['kernel']}: {roof['avg_launch_ms']:.3f} ms avg, "
        f"{roof['achieved']:.0f} GB/s")
    log(f"[neumann512] dominant kernel (f64) {roof64['kernel']}: {roof64['avg_launch_ms']:.3f} ms avg, "
        f"{roof64['achieved']:.0f} GB/s")
    out = base_record(args, "grid points solved/s (FP32+FP64 refinement to 1e-12 rel. error), with HBM GB/s",
                      npts / (ms_r * 1e-3), "points/s", ms_r, "f32+f64",
                      {"workload": f"neumann_vertex_{n}^3_dct1_fd_blobs64", "shape": list(d["shape"]),
                       "bc": "N,N,N (vertex)", "approx": "fd", "refine_corrections": args.max_iter})
    out["hbm_gbs_step"] = step_gbs(rec_r, reps, ms_r)
    out["fp64_path"] = {"points_per_s": npts / (ms_64 * 1e-3), "ms_per_solve": ms_64,
                        "hbm_gbs_step": step_gbs(rec_64, reps, ms_64),
                        "speed_ratio_f32r_over_f64": ms_64 / ms_r, "roofline": roof64}
    out["rel_resid"] = {"f32r": info_r["rel_resid"], "f64": info_64["rel_resid"]}
    out["roofline"] = roof
    out["wall_ms_per_step"] = wall_r
    if not args.no_cpu:
        log("[neumann512] running the CPU oracle on the same input (one full solve)")
        ref, dt, threads = cpu_oracle(d, g)
        err_r, err_64 = rel(phi_r, ref), rel(phi_64, ref)
        log(f"[neumann512] oracle {dt:.1f} s; rel err f32r {err_r:.3e}, f64 {err_64:.3e}")
        out["cpu_baseline"] = {"value": npts / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
                               "sample": f"one full {n}^3 solve of the same input (dense FP64 transform "
                                         f"matrices, {dt:.1f} s)"}
        out["rel_err_vs_oracle"] = {"f32r": err_r, "f64": err_64}
    plan_r.close()
    plan_64.close()
    return out


def run_periodic32(args):
    import torch
    import workloads
    import paper_1409_8116_amd as mp
    d, g = workloads.periodic_noise(32, seed=1)
    npts = int(np.prod(d["shape"]))
    rhs = torch.tensor(g, dtype=torch.float64, device="cuda")
    phi = torch.empty_like(rhs)
    eager = mp.Plan.from_desc(d, prec="f64")
    graph = mp.Plan.from_desc(d, prec="f64", graph=True)
    steps = max(args.steps, 1000)
    ms_e, _ = timed(lambda: eager.solve(rhs, phi), steps, 50)
    phi_g = torch.empty_like(rhs)
    ms_g, _ = timed(lambda: graph.solve(rhs, phi_g), steps, 50)
    log(f"[periodic32] {ms_e * 1e3:.1f} us eager, {ms_g * 1e3:.1f} us graph-replayed")
    recs, reps = profile_plan(lambda: mp.Plan.from_desc(d, prec="f64", profile=True), rhs)
    out = {"workload": "periodic_32^3_fd_fp64", "ms_per_solve": ms_g, "points_per_s": npts / (ms_g * 1e-3),
           "us_per_solve": {"eager": ms_e * 1e3, "graph": ms_g * 1e3},
           "hbm_gbs_step": step_gbs(recs, reps, ms_g), "roofline": kernel_roofline(recs, reps),
           "note": "launch-latency bound; 2.6 MB per solve stays in cache, so GB/s is not an HBM figure"}
    if not args.no_cpu:
        ref, dt, threads = cpu_oracle(d, g)
        out["rel_err_vs_oracle"] = {"eager": rel(phi, ref), "graph": rel(phi_g, ref)}
        out["cpu_baseline"] = {"value": npts / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
                               "sample": "one 32^3 solve"}
    eager.close()
    graph.close()
    return out


def run_mixed256(args):
    import torch
    import workloads
    import paper_1409_8116_amd as mp
    outs = {}
    for approx in ("fd", "ps"):
        d, g, _ = workloads.mixed_modes(256, seed=2, approx=approx)
        npts = int(np.prod(d["shape"]))
        ref = None
        if not args.no_cpu:
            ref, dt, threads = cpu_oracle(d, g)
        for prec in ("f64", "f32"):
            dt_ = torch.float64 if prec == "f64" else torch.float32
            rhs = torch.tensor(g, dtype=dt_, device="cuda")
            phi = torch.empty_like(rhs)
            plan = mp.Plan.from_desc(d, prec=prec)
            ms, _ = timed(lambda: plan.solve(rhs, phi), args.steps, args.warmup)
            recs, reps = profile_plan(lambda: mp.Plan.from_desc(d, prec=prec, profile=True), rhs)
            o = {"workload": f"mixed_256^3_P-Ds-Ns_{approx}_{prec}", "ms_per_solve": ms,
                 "points_per_s": npts / (ms * 1e-3), "hbm_gbs_step": step_gbs(recs, reps, ms),
                 "roofline": kernel_roofline(recs, reps)}
            if ref is not None:
                o["rel_err_vs_oracle"] = rel(phi, ref)
                o["cpu_baseline"] = {"value": npts / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
                                     "sample": f"one 256^3 {approx} solve"}
            log(f"[mixed256] {approx} {prec}: {ms:.3f} ms, {o['hbm_gbs_step']:.0f} GB/s"
                + (f", rel err {o['rel_err_vs_oracle']:.2e}" if ref is not None else ""))
            outs[f"{approx}_{prec}"] = o
            plan.close()
    return outs


def run_batch(args):
    import torch
    import workloads
    import paper_1409_8116_amd as mp
    descs = workloads.batch_2d(count=2048, seed=4)
    npts = sum(int(np.prod(d["shape"])) for d in descs)
    log(f"[batch2048] 2048 grids, {npts:.3e} points; generating right-hand sides")
    rhs = [torch.tensor(workloads.batch_rhs(d, i), dtype=torch.float64, device="cuda") for i, d in enumerate(descs)]
    phi = [torch.empty_like(r) for r in rhs]
    t0 = time.perf_counter()
    plan = mp.BatchPlan(descs, prec="f32r", max_iter=args.max_iter, tune=True)
    tplan = time.perf_counter() - t0
    log(f"[batch2048] tuned batch plan built in {tplan:.1f} s")
    ms, _ = timed(lambda: plan.solve(rhs, phi), args.steps, args.warmup)
    info = plan.info()
    # algorithmic bytes: 2D F32R with K corrections, 32 + 64 K bytes per point (unfused model)
    gbs = npts * (32 + 64 * args.max_iter) / (ms * 1e-3) / 1e9
    out = {"workload": "batch_2048x2D_64-1024_f32r_tuned", "grids": 2048, "points": npts, "ms_per_step": ms,
           "points_per_s": npts / (ms * 1e-3), "hbm_gbs_model": gbs, "plan_build_s": tplan,
           "rel_resid_worst": info["rel_resid"]}
    log(f"[batch2048] {ms:.2f} ms per batch, worst rel resid {info['rel_resid']:.2e}")
    if not args.no_cpu:
        worst, tsum, nsub, threads = 0.0, 0.0, 0, 1
        for i in range(0, 2048, 32):
            d = descs[i]
            ref, dt, threads = cpu_oracle(d, rhs[i].cpu().numpy())
            worst = max(worst, rel(phi[i], ref))
            tsum += dt
            nsub += int(np.prod(d["shape"]))
        out["rel_err_vs_oracle_subset64"] = worst
        out["cpu_baseline"] = {"value": nsub / tsum, "unit": "points/s", "cores": threads, "kind": "oracle",
                               "sample": "64 of the 2048 grids (every 32nd)"}
        log(f"[batch2048] worst rel err over 64 grids {worst:.2e}")
    plan.close()
    return out


def run_channel(args):
    import torch
    import workloads
    import paper_1409_8116_amd as mp
    d = workloads.channel_desc()
    npts = int(np.prod(d["shape"]))
    nrhs = args.nrhs
    plan = mp.Plan.from_desc(d, prec="f32r", max_iter=args.max_iter, graph=True)
    rhs = torch.empty(d["shape"], dtype=torch.float64, device="cuda")
    phi = torch.empty_like(rhs)
    # the graph is captured for this (rhs, phi) pair; each step regenerates rhs in place
    g0 = workloads.channel_divergence(d, 0, device="cuda")
    rhs.copy_(g0)
    plan.solve(rhs, phi)
    torch.cuda.synchronize()
    first = phi.clone()
    total = 0.0
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    worst_resid = 0.0
    for s in range(nrhs):
        rhs.copy_(workloads.channel_divergence(d, s, device="cuda"))
        start.record()
        plan.solve(rhs, phi)
        end.record()
        torch.cuda.synchronize()
        total += start.elapsed_time(end)
        if s % 50 == 0 or s == nrhs - 1:
            worst_resid = max(worst_resid, plan.info()["rel_resid"])
    ms = total / nrhs
    recs, reps = profile_plan(lambda: mp.Plan.from_desc(d, prec="f32r", max_iter=args.max_iter, profile=True), rhs)
    out = {"workload": f"channel_1024x512x256_P-Ns-P_graph_f32r_{nrhs}rhs", "ms_per_rhs": ms,
           "refine_corrections": args.max_iter,
           "points_per_s": npts / (ms * 1e-3), "hbm_gbs_step": step_gbs(recs, reps, ms),
           "roofline": kernel_roofline(recs, reps), "rel_resid_worst_sampled": worst_resid}
    log(f"[channel] {ms:.3f} ms per right-hand side, {out['hbm_gbs_step']:.0f} GB/s")
    # the plain FP64 path on the same stream buffer, for comparison
    plan64 = mp.Plan.from_desc(d, prec="f64")
    phi64 = torch.empty_like(rhs)
    ms64, _ = timed(lambda: plan64.solve(rhs, phi64), max(args.steps, 10), args.warmup)
    plan64.close()
    out["fp64_ms_per_rhs"] = ms64
    log(f"[channel] FP64 path {ms64:.3f} ms per right-hand side")
    if not args.no_cpu:
        ref, dt, threads = cpu_oracle(d, g0.cpu().numpy())
        out["rel_err_vs_oracle_rhs0"] = rel(first, ref)
        out["cpu_baseline"] = {"value": npts / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
                               "sample": "one 1024x512x256 solve (rhs #0)"}
        log(f"[channel] rel err rhs #0 {out['rel_err_vs_oracle_rhs0']:.2e}")
    plan.close()
    return out


def run_projection(args):
    """One projection step of the channel flow (Section 5.1) per step: the
    divergence of a staggered velocity, the solve and the velocity / pressure
    correction, FP64 (fused into the first and last line passes) and FP32 +
    refinement, next to the plain solve of the same grid."""
    import torch
    import workloads
    import paper_1409_8116_amd as mp
    d = workloads.channel_desc()
    d = dict(d, grid=("s", "s", "s"))
    shape = d["shape"]
    npts = int(np.prod(shape))
    log("[projection] generating the staggered velocity")
    vel0 = workloads.mac_velocity(d, seed=9)
    p0 = np.random.default_rng(10).standard_normal(shape)
    vel = [torch.tensor(u, device="cuda") for u in vel0]
    p = torch.tensor(p0, device="cuda")
    phi = torch.empty_like(p)
    work = [torch.empty_like(u) for u in vel]
    pw = torch.empty_like(p)
    adt = 0.02
    out = {"workload": "projection_1024x512x256_P-Ns-P_staggered"}

    def step(plan):
        for w, u in zip(work, vel):
            w.copy_(u)
        pw.copy_(p)
        plan.project(work, pw, adt, phi)

    # the copies that restore u* and p each step are timed on their own and removed
    copy_ms, _ = timed(lambda: ([w.copy_(u) for w, u in zip(work, vel)], pw.copy_(p)), args.steps, args.warmup)
    # algorithmic bytes per point of the fused FP64 step: pass 1 reads three
    # velocity components and writes phi (32), three middle passes (48), the
    # last pass reads phi, p, w and writes them (48), the u / v correction
    # reads phi, u, v and writes u, v (40)
    fused_bytes = 168.0
    for prec, k in (("f64", 0), ("f32r", args.max_iter)):
        plan = mp.Plan.from_desc(d, prec=prec, max_iter=max(k, 1))
        ms, _ = timed(lambda: step(plan), args.steps, args.warmup)
        ms -= copy_ms
        solve_ms, _ = timed(lambda: plan.solve(pw, phi), args.steps, args.warmup)
        rec = {"ms_per_step": ms, "points_per_s": npts / (ms * 1e-3), "plain_solve_ms": solve_ms}
        if prec == "f64":
            rec["hbm_gbs_step"] = npts * fused_bytes / (ms * 1e-3) / 1e9
        else:
            rec["refine_corrections"] = k
        step(plan)
        torch.cuda.synchronize()
        if prec == "f32r":
            rec["rel_resid"] = plan.info()["rel_resid"]
        out[prec] = rec
        log(f"[projection] {prec}: {ms:.3f} ms per step (plain solve {solve_ms:.3f} ms)")
        plan.close()
    if not args.no_cpu:
        import oracle
        axes = oracle.axes_from(shape, d["h"], d["bc"], d["grid"])
        t0 = time.perf_counter()
        rv, rp, rphi = oracle.projection_step(vel0, p0, axes, adt)
        dt = time.perf_counter() - t0
        out["rel_err_vs_oracle_f32r"] = {
            "phi": rel(phi, rphi),
            "velocity": max(float(np.linalg.norm(w.cpu().numpy() - r) / np.linalg.norm(u))
                            for w, r, u in zip(work, rv, vel0))}
        out["cpu_baseline"] = {"value": npts / dt, "unit": "points/s", "cores": cpu_threads(), "kind": "oracle",
                               "sample": "one projection step of the same field"}
        log(f"[projection] oracle {dt:.1f} s, rel err phi {out['rel_err_vs_oracle_f32r']['phi']:.2e}")
    return out


def run_copy(args):
    """A device copy of known size: the FETCH_SIZE / WRITE_SIZE counters it reads,
    divided by its bytes, scale the counters of the solver kernels."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    ms, _ = timed(lambda: dst.copy_(src), max(args.steps, 3), 1)
    return {"workload": "copy_1GiB", "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


SECONDARY = {"periodic32": run_periodic32, "mixed256": run_mixed256, "batch2048": run_batch,
             "channel": run_channel, "projection": run_projection}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all",
                    choices=["all", "neumann512", "copy"] + sorted(SECONDARY))
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--max-iter", type=int, default=2)
    ap.add_argument("--nrhs", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--f64-arith", action="store_true",
                    help="refinement plans compute the transforms in FP64 on FP32-stored data")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver build has no multi-GPU path "
              "(the slab decomposition over RCCL is described, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "copy":
        print(json.dumps(run_copy(args)), flush=True)
        return
    if args.workload in SECONDARY:
        print(json.dumps(SECONDARY[args.workload](args)), flush=True)
        return
    rec = run_neumann(args)
    if args.workload == "all":
        rec["configs"] = {}
        for name, fn in SECONDARY.items():
            log(f"--- {name}")
            t0 = time.perf_counter()
            rec["configs"][name] = fn(args)
            log(f"--- {name} done in {time.perf_counter() - t0:.1f} s")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
