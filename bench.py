#!/usr/bin/env python3
"""Throughput of the thin-disk force solve on one MI355X.

One step = one full force solve (every pass of the hot path) of the workload:
  two nested levels of 256 x 256 cells, ratio 2, the fine level covering the
  central [-1/2,1/2]^2 of the [-1,1]^2 base; sigma = Maclaurin disk R = 0.8
  plus a Gaussian clump (amplitude 5, width 0.03) at (0.2, 0.1); sigma in,
  the in-cell slopes estimated from it inside the solve (centred
  differences, one-sided at patch edges; --slopes given passes central
  differences of the analytic sigma instead); FP32 FFT passes with
  FP64-built kernel spectra.
Inputs are resident in HBM before the timed region; kernel spectra are
resident (plan built beforehand).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]
                  [--workload two-level-256|single-64|four-level-512|example3-512|
                              example1-1024|batch-64|serve]
                  [--mode eager|graph] [--slopes estimate|given]
                  [--quantity force|potential] [--no-cpu] [--tune DB]

Other workloads: batch-64 = 64 independent disks (base N in {64..512}, 1-3
nested levels, random aligned refinement, generalized Maclaurin sigma) solved
by one batched launch set per step; serve = Poisson arrivals (mean rate
--rate) of mixed hierarchies (base N in {128..1024}, 1-5 levels) into the
serving loop, reporting p50/p99 latency beside throughput.
"""
import argparse
import contextlib
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "force-solve cells/s at rel-L2 <=1e-5 vs FP64 oracle; p50/p99 latency"

# HBM bytes per launch of a pass, from rocprofv3 FETCH_SIZE + WRITE_SIZE runs
# of this script, each scaled by the ratio of a plain copy kernel's known
# bytes to what the same counter read for it.  Keyed by (workload, dtype,
# slopes mode, pass) and tied to the SHA-256 of the sources they were taken
# on -- the kernels and the plan builder, whose jobs and launch shapes
# decide the traffic too: a changed source reports null until it is
# profiled again.
TRAFFIC = {
    ("two-level-256", "f32", "estimate", "col"): (35638059, "11647acb5d2dd52a"),
    ("two-level-256", "f32", "estimate", "row_inv"): (5485122, "11647acb5d2dd52a"),
    ("two-level-256", "f32", "estimate", "row_fwd"): (9355045, "11647acb5d2dd52a"),
}


@contextlib.contextmanager
def gc_paused():
    """Python's cyclic garbage collector paused for a timed loop, as timeit
    does: a full collection stalls the submitting thread for milliseconds
    while only a few solves are queued on the device, and the GPU idles
    (2000 eager two-level solves: 67-69 us each with it, 52.5 us without)."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("td_kernels.hip", "td_fft.hpp", "td_jobs.h", "td_launch.h", "td_api.cpp"):
        with open(os.path.join(ROOT, "paper_1603_03142_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, dtype, slopes, pass_name):
    rec = TRAFFIC.get((workload_name, dtype, slopes, pass_name))
    if rec is None or rec[1] != kernel_source_hash():
        return None
    return rec[0]


def copy_calibration(torch, mb):
    """A plain device copy of known size (mb MiB read + mb MiB written), run
    outside the timed region, for scaling HBM byte counters."""
    n = (mb << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def workload(name):
    import synth
    if name == "two-level-256":
        hier, fn = synth.config2()
    elif name == "single-64":
        hier, fn = synth.config1()
    elif name == "four-level-512":
        hier, fn = synth.config3()
    elif name == "example3-512":
        # the paper's Example 3: two sigma_D5 disks, two level-1 patches
        hier, fn = synth.example_hierarchy(3, 512), synth.two_disks()
    elif name == "example1-1024":
        # the paper's Example 1 at its largest size (convergence study)
        hier, fn = synth.example_hierarchy(1, 1024), synth.disk_dn(5, 0.85)
    else:
        raise SystemExit(f"unknown workload {name}")
    return hier, fn


def host_fields(synth, hier, fn, slopes):
    """sigma per patch, and the slope fields when they are passed in."""
    if slopes == "estimate":
        s, _, _ = synth.sample_fields(hier, fn, "none")
        return s, None, None
    return synth.sample_fields(hier, fn, "central")


def dev_fields(torch, tdt, arrs, slopes):
    dev = lambda a: None if a is None else [torch.as_tensor(x, dtype=tdt, device="cuda")
                                            for x in a]
    return (*[dev(a) for a in arrs], slopes)


def run_batch(args, td, torch, synth):
    """64 independent hierarchies per step, one batched launch set."""
    import numpy as np
    disks = synth.config4(seed=4, count=64)
    ctx = td.Context(0)
    if args.tune:
        ctx.autotune(args.dtype, 1024, args.tune)
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    plans, fields = [], []
    for hier, fn in disks:
        plans.append(ctx.plan(hier, args.dtype))
        fields.append(dev_fields(torch, tdt, host_fields(synth, hier, fn, args.slopes),
                                 args.slopes))
    batch = td.Batch(ctx, plans)
    outs = [p.outputs() for p in plans]
    use_graph = args.mode == "graph"
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.solve(fields, outs, use_graph=use_graph, stream=stream)
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.solve(fields, outs, use_graph=use_graph, stream=stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    cells = sum(p.cells for p in plans)
    return {
        "metric": METRIC,
        "value": cells * args.steps / el, "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "batch-64", "hierarchies": len(plans), "cells_per_step": cells,
                   "mode": args.mode, "slopes": args.slopes,
                   "workspace_bytes": batch.footprint(), "python_gc": "paused in timed loops"},
        "roofline": None, "cpu_baseline": None,
    }


def run_serve(args, td, torch, synth):
    """Poisson arrivals of mixed hierarchies into the serving loop."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(5))
    reqs = synth.config5_requests(seed=5, rate=args.rate, duration=args.duration)
    ctx = td.Context(0, hbm_budget=int(args.budget_gb * (1 << 30)))
    if args.tune:
        ctx.autotune(args.dtype, 2048, args.tune)
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    # request types: distinct hierarchies planned once (kernel spectra and job
    # lists resident); every arrival draws one type
    ntypes = args.types
    types = []
    log = lambda msg: print(f"[serve] {msg}", file=sys.stderr, flush=True)
    tp = time.perf_counter()
    for k in range(ntypes):
        _, hier, (order, alpha, fseed) = reqs[k % len(reqs)]
        fn = synth.request_sigma(order, alpha, fseed, hier.h0)
        plan = ctx.plan(hier, args.dtype)
        outs = [plan.outputs() for _ in range(2)]
        types.append((plan, dev_fields(torch, tdt, host_fields(synth, hier, fn, args.slopes),
                                       args.slopes), outs))
        log(f"planned type {k}: levels {len(hier.patches)} n {hier.patches[0].n} "
            f"workspace {plan.footprint()[0] / 2**30:.2f} GiB ({time.perf_counter() - tp:.1f} s)")
    srv = td.Server(ctx, max_inflight=args.inflight, max_batch=args.max_batch)
    srv.set_queue_limit(args.queue_limit)
    # warm-up: each type once
    for plan, f, outs in types:
        srv.submit(plan, *f[:3], *outs[0], slopes=f[3])
        srv.drain()
    log(f"warm-up done ({time.perf_counter() - tp:.1f} s)")
    torch.cuda.synchronize()
    st0 = srv.stats()
    arrivals = [t for t, _, _ in reqs]
    pick = rng.integers(0, ntypes, len(arrivals))
    tickets = []
    refused = 0
    t0 = time.perf_counter()
    next_log = 1.0
    for k, ta in enumerate(arrivals):
        while time.perf_counter() - t0 < ta:
            pass
        plan, f, outs = types[pick[k]]
        try:
            tk, _, _ = srv.submit(plan, *f[:3], *outs[k % 2], queue_if_full=False,
                                  slopes=f[3])
            tickets.append((tk, plan.cells))
        except td.TdError as e:
            if e.status != 6:  # TD_EBUSY: the bounded queue is full
                raise
            refused += 1
        if ta >= next_log:
            log(f"t={ta:.1f} s: {len(tickets)} admitted, {refused} refused, "
                f"{srv.stats()['completed'] - st0['completed']} completed")
            next_log += 1.0
    t_arr = time.perf_counter() - t0
    log(f"{len(tickets)} requests admitted, {refused} refused ({t_arr:.2f} s)")
    last = time.perf_counter()
    while True:
        n_done = sum(srv.poll(tk)[0] for tk, _ in tickets[::max(1, len(tickets) // 200)])
        if n_done == len(tickets[::max(1, len(tickets) // 200)]):
            break
        if time.perf_counter() - last > 5:
            log(f"draining: {srv.stats()['completed']} completed "
                f"({time.perf_counter() - t0:.1f} s)")
            last = time.perf_counter()
        time.sleep(0.01)
    srv.drain()
    el = time.perf_counter() - t0
    lats = []
    cells = 0
    for tk, c in tickets:
        done, lat = srv.poll(tk)
        assert done
        lats.append(lat)
        cells += c
    st = srv.stats()
    st = {k: st[k] - st0[k] if k != "peak_queue" else st[k] for k in st}
    lats = np.array(lats)
    srv.close()
    return {
        "metric": METRIC,
        "value": cells / el, "unit": "cells/s", "n_gpus": 1, "steps": len(tickets),
        "warmup": ntypes, "ms_per_step": 1000 * el / len(tickets), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "serve", "offered_rate": args.rate, "duration_s": args.duration,
                   "request_types": ntypes, "max_inflight": args.inflight,
                   "max_batch": args.max_batch, "queue_limit": args.queue_limit,
                   "hbm_budget_gb": args.budget_gb, "slopes": args.slopes},
        "serving": {"offered": len(arrivals), "admitted": len(tickets), "refused": refused,
                    "arrival_window_s": t_arr, "wall_s": el,
                    "sustained_req_per_s": len(tickets) / el,
                    "p50_ms": float(np.percentile(lats, 50) * 1e3),
                    "p99_ms": float(np.percentile(lats, 99) * 1e3),
                    "mean_ms": float(lats.mean() * 1e3), **st},
        "roofline": None, "cpu_baseline": None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="two-level-256")
    ap.add_argument("--mode", default="eager", choices=["eager", "graph"])
    ap.add_argument("--quantity", default="force", choices=["force", "potential"],
                    help="force (the metric) or the potential (a TD_POTENTIAL plan)")
    ap.add_argument("--slopes", default="estimate", choices=["estimate", "given"],
                    help="estimate: sigma in, slopes from it inside the solve; given: "
                         "central differences of the analytic sigma passed in")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tune", metavar="DB", default=None,
                    help="autotune launch shapes first (JSON-lines database path)")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: mean arrivals per s")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals")
    ap.add_argument("--queue-limit", type=int, default=256,
                    help="serve: requests waiting for admission at most (others refused)")
    ap.add_argument("--types", type=int, default=48, help="serve: distinct request hierarchies")
    ap.add_argument("--inflight", type=int, default=4, help="serve: concurrent batches")
    ap.add_argument("--max-batch", type=int, default=16, help="serve: requests per batch")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: HBM budget (GiB)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run a plain copy of this many MiB first (counter calibration)")
    ap.add_argument("--no-fp64-leg", action="store_true",
                    help="skip the per-solve FP64 eager comparison")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs the solver on a single "
              "MI355X (multi-GPU sharding is design-only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1603_03142_amd as td
    import synth

    torch.cuda.set_device(0)
    if args.copy_mb:
        copy_calibration(torch, args.copy_mb)
    if args.workload in ("batch-64", "serve"):
        out = (run_batch if args.workload == "batch-64" else run_serve)(args, td, torch, synth)
        print(json.dumps(out), flush=True)
        return
    hier, fn = workload(args.workload)
    sig, dx, dy = host_fields(synth, hier, fn, args.slopes)
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    S, DX, DY, SL = dev_fields(torch, tdt, (sig, dx, dy), args.slopes)

    ctx = td.Context(0)
    tune_s = None
    if args.tune:
        t0 = time.perf_counter()
        ctx.autotune(args.dtype, max(p.n for p in hier.patches) * 2, args.tune)
        tune_s = round(time.perf_counter() - t0, 2)
    t0 = time.perf_counter()
    plan = ctx.plan(hier, args.dtype, quantity=args.quantity)
    plan_s = time.perf_counter() - t0
    FX, FY = plan.outputs()  # FY is None for a potential plan (Phi in FX)
    cells = plan.cells
    stream = torch.cuda.current_stream()

    if args.mode == "graph":
        batch = td.Batch(ctx, [plan])
        step = lambda: batch.solve([(S, DX, DY, SL)], [(FX, FY)], use_graph=True, stream=stream)
    else:
        step = lambda: plan.solve(S, DX, DY, FX, FY, stream=stream, slopes=SL)

    # warm-up: the first solve untimed (first launches load code objects,
    # and a profiler sets up its tracing then), the others with every pass
    # timed (eager): per-pass breakdown and the dominant pass, which alone is
    # timed over the measured region
    warm = None
    n_first = 1 if args.warmup > 1 else 0
    for _ in range(n_first):
        step()
    torch.cuda.synchronize()
    ctx.timing(args.mode == "eager")
    ctx.timing_read()
    for _ in range(args.warmup - n_first):
        step()
    torch.cuda.synchronize()
    if args.mode == "eager" and args.warmup > 0:
        warm = ctx.timing_read()
    ctx.timing(False)
    dom = max(warm, key=lambda p: warm[p][0]) if warm else None
    if dom:
        ctx.timing(True, passes=[dom])
        ctx.timing_read()  # clear
    torch.cuda.synchronize()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    elapsed = t1 - t0
    passes = ctx.timing_read() if dom else None
    ctx.timing(False)
    ms_per_step = 1000.0 * elapsed / args.steps
    value = cells * args.steps / elapsed

    # latency of one solve on an idle device: enqueue to completion, each
    # solve synchronised (after the timed region, so it does not change it)
    lat = []
    with gc_paused():
        for _ in range(max(50, min(400, args.steps))):
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
    lat = np.array(lat) * 1e3
    latency = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "samples": len(lat),
               "how": "single solves, each from enqueue to completion (host clock), device idle"}

    # roofline of the dominant pass (algorithmic bytes / mean launch time)
    roof = None
    traffic = plan.traffic(args.slopes)
    if passes:
        ms, launches = passes[dom]
        per_launch_s = ms / 1000.0 / max(launches, 1)
        launches_per_solve = launches / args.steps
        bytes_per_launch = traffic[dom] / max(launches_per_solve, 1e-30)
        achieved = bytes_per_launch / per_launch_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (measured_traffic(args.workload, args.dtype, args.slopes, dom)
                            if args.quantity == "force" else None),
                "avg_launch_us": round(per_launch_s * 1e6, 2),
                "alg_bytes_per_launch": int(bytes_per_launch),
                "passes_us_per_solve_warmup": {p: round(1000.0 * warm[p][0] / (args.warmup - n_first), 2)
                                               for p in warm}}

    # the plain per-solve FP64 GPU path (eager, one solve per call, FP64
    # throughout) on the same workload, for the speed-up of this run over it
    fp64 = None
    if not args.no_fp64_leg and not (args.dtype == "f64" and args.mode == "eager"):
        S64, DX64, DY64, _ = dev_fields(torch, torch.float64, (sig, dx, dy), args.slopes)
        ctx64 = td.Context(0)
        plan64 = ctx64.plan(hier, "f64", quantity=args.quantity)
        FX64, FY64 = plan64.outputs()
        k64 = max(3, args.steps // 4)
        for _ in range(3):
            plan64.solve(S64, DX64, DY64, FX64, FY64, stream=stream, slopes=SL)
        torch.cuda.synchronize()
        with gc_paused():
            t0 = time.perf_counter()
            for _ in range(k64):
                plan64.solve(S64, DX64, DY64, FX64, FY64, stream=stream, slopes=SL)
            torch.cuda.synchronize()
            el64 = time.perf_counter() - t0
        v64 = cells * k64 / el64
        fp64 = {"value": v64, "unit": "cells/s", "steps": k64,
                "ms_per_step": 1000.0 * el64 / k64, "speedup": value / v64}
        plan64.close()
        ctx64.close()
        del S64, DX64, DY64, FX64, FY64

    # CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    acc = None
    if not args.no_cpu:
        import oracle
        if args.slopes == "estimate":
            dx, dy = oracle.slopes(hier, sig)
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        # a probe of 64 targets (a smaller one overestimates the per-target
        # time: the thread pool starts up inside it)
        pot = args.quantity == "potential"
        direct = oracle.potential if pot else oracle.forces
        probe = synth.sample_targets(hier, 64, seed=1)
        tp0 = time.perf_counter()
        direct(hier, sig, dx, dy, probe, nthreads=nthreads)
        per_target = (time.perf_counter() - tp0) / len(probe[0])
        count = max(8, min(4096, int(args.cpu_seconds / max(per_target, 1e-9))))
        tg = synth.sample_targets(hier, count, seed=2)
        tp0 = time.perf_counter()
        ref = direct(hier, sig, dx, dy, tg, nthreads=nthreads)
        ox, oy = (ref, np.zeros_like(ref)) if pot else ref
        cpu_s = time.perf_counter() - tp0
        model = None
        try:
            with open("/proc/cpuinfo") as f:
                model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                             None)
        except OSError:
            pass
        cpu = {"value": round(len(tg[0]) / cpu_s, 2), "unit": "cells/s", "cores": nthreads,
               "kind": "oracle", "cpu_model": model,
               "full_solve_s_extrapolated": round(cells * cpu_s / len(tg[0]), 1),
               "sample": f"{len(tg[0])} sampled target cells of the workload (25% within 2 "
                         f"cells of a level interface), each summed over every active source "
                         f"cell; {cpu_s:.1f} s"}
        fxc = [f.double().cpu().numpy() for f in FX]
        gx = np.array([fxc[p][j, i] for p, i, j in zip(*tg)])
        if pot:
            gy = np.zeros_like(gx)
        else:
            fyc = [f.double().cpu().numpy() for f in FY]
            gy = np.array([fyc[p][j, i] for p, i, j in zip(*tg)])
        acc = math.sqrt((((gx - ox) ** 2).sum() + ((gy - oy) ** 2).sum()) /
                        ((ox ** 2).sum() + (oy ** 2).sum()))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "levels": hier.nlevels,
                   "patches": [[p.level, p.n] for p in hier.patches], "ratio": hier.ratio,
                   "cells_per_solve": cells, "mode": args.mode, "slopes": args.slopes,
                   "quantity": args.quantity,
                   "plan_build_s": round(plan_s, 3), "autotune_s": tune_s,
                   "python_gc": "paused in timed loops"},
        "latency": latency,
        "roofline": roof,
        "cpu_baseline": cpu,
        "rel_l2_vs_oracle_sampled": acc,
        "fp64_per_solve_gpu": fp64,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
