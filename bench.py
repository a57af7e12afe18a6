#!/usr/bin/env python3
"""Throughput of the thin-disk force solve on one MI355X.

One step = one full force solve (every pass of the hot path) of the workload,
by default four nested levels of 512 x 512 cells (ratio 2, level-l extent
2^(1-l), centred as near (0.3, 0) as the lattices allow); sigma = generalized
Maclaurin disk (1 - r^2/0.81)^(3/2) times a seeded lognormal perturbation
(std 0.2, correlation length 4 base cells); the in-cell slopes are central
differences of the analytic sigma at x +- h, computed on the host in FP64 and
handed identically to the oracle and the GPU (rounded to FP32 for the FP32
path); FP32 FFT passes with FP64-built kernel spectra.  Inputs are resident in
HBM before the timed region; kernel spectra are resident (plan built
beforehand).  Prints one JSON line, which also carries:
  * slopes_estimate: the same workload with sigma in and the slopes estimated
    inside the solve;
  * fp64_per_solve_gpu: the plain per-solve FP64 GPU path (speed-up, and its
    error against the oracle on the sampled targets);
  * cpu_baseline: the oracle on a bounded sample of stratified targets, with
    the FP32 result's rel-L2 against it, overall and per level;
  * serving: Poisson arrivals of mixed hierarchies at --rate into the serving
    loop (p50 / p99 latency, sustained requests/s, refusals, deferrals).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]
                  [--workload four-level-512|two-level-256|single-64|example3-512|
                              example1-1024|batch-64|serve]
                  [--mode eager|graph] [--slopes given|estimate]
                  [--quantity force|potential] [--no-cpu] [--no-serve] [--tune DB]
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
DEFAULT_WORKLOAD = "four-level-512"

# HBM bytes per launch of a pass, from rocprofv3 FETCH_SIZE + WRITE_SIZE runs
# of this script, each scaled by the ratio of a copy kernel's known bytes to
# what the same counter read for it.  Keyed by (workload, dtype, slopes mode,
# pass) and tied to the SHA-256 of the sources they were taken on -- the
# kernels and the plan builder, whose jobs and launch shapes decide the
# traffic too: a changed source reports null until it is profiled again.
TRAFFIC = {
    ("four-level-512", "f32", "given", "row_fwd"): (244308064, "c537993581510c47"),
    ("four-level-512", "f32", "given", "col"): (1709918767, "c537993581510c47"),
    ("four-level-512", "f32", "given", "row_inv"): (152142150, "c537993581510c47"),
}


@contextlib.contextmanager
def gc_paused():
    """Python's cyclic garbage collector paused for a timed loop, as timeit
    does: a full collection stalls the submitting thread for milliseconds
    while only a few solves are queued on the device, and the GPU idles."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
    """Plain device copies of known size, run outside the timed region, for
    scaling HBM byte counters: a torch copy (16-byte accesses) and an
    element-wise float64 add of two operands (8-byte accesses, the width of
    the solve's complex FP32 gathers), mb MiB per operand."""
    n = (mb << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    a64 = a.view(torch.float64)
    b64 = b.view(torch.float64)
    for _ in range(3):
        torch.add(a64, 1.0, out=b64)
    torch.cuda.synchronize()
    del a, b, a64, b64


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
    """sigma per patch, and the slope fields when they are passed in (central
    differences of the analytic sigma at x +- h, host FP64)."""
    if slopes == "estimate":
        s, _, _ = synth.sample_fields(hier, fn, "none")
        return s, None, None
    return synth.sample_fields(hier, fn, "central")


def dev_fields(torch, tdt, arrs, slopes):
    dev = lambda a: None if a is None else [torch.as_tensor(x, dtype=tdt, device="cuda")
                                            for x in a]
    return (*[dev(a) for a in arrs], slopes)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                        None)
    except OSError:
        return None


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()


def sampled_values(fields, targets):
    """Values of per-patch device arrays at (patch, i, j) targets, as float64."""
    import numpy as np
    host = [f.double().cpu().numpy() for f in fields]
    return np.array([host[p][j, i] for p, i, j in zip(*targets)])


def errors(hier, targets, gx, gy, ox, oy):
    """rel-L2 over (Fx, Fy), overall and per level, and the largest absolute
    error, of sampled values against the oracle's."""
    import numpy as np

    def rel(s):
        num = ((gx[s] - ox[s]) ** 2).sum() + ((gy[s] - oy[s]) ** 2).sum()
        den = (ox[s] ** 2).sum() + (oy[s] ** 2).sum()
        return float(math.sqrt(num / den)) if den > 0 else 0.0
    lev = np.array([hier.patches[p].level for p in targets[0]])
    return {"rel_l2": rel(np.ones(len(gx), bool)),
            "rel_l2_per_level": {str(l): rel(lev == l) for l in sorted(set(lev.tolist()))},
            "max_abs": float(max(np.abs(gx - ox).max(), np.abs(gy - oy).max())),
            "targets": int(len(gx))}


def oracle_sample(hier, sig, dx, dy, seconds, potential=False, seed=2):
    """The oracle on stratified targets (25% within 2 cells of a level
    interface), as many as fit in about `seconds` of the host's cores; a
    64-target probe sizes the sample.  Returns (targets, ox, oy, info)."""
    import numpy as np
    import oracle
    import synth
    nthreads = oracle_threads()
    direct = oracle.potential if potential else oracle.forces
    probe = synth.sample_targets(hier, 64, seed=1)
    t0 = time.perf_counter()
    direct(hier, sig, dx, dy, probe, nthreads=nthreads)
    per_target = (time.perf_counter() - t0) / len(probe[0])
    count = max(8 * len(hier.patches), min(4096, int(seconds / max(per_target, 1e-9))))
    tg = synth.sample_targets(hier, count, seed=seed)
    t0 = time.perf_counter()
    ref = direct(hier, sig, dx, dy, tg, nthreads=nthreads)
    cpu_s = time.perf_counter() - t0
    ox, oy = (ref, np.zeros_like(ref)) if potential else ref
    info = {"value": round(len(tg[0]) / cpu_s, 2), "unit": "cells/s", "cores": nthreads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "full_solve_s_extrapolated": round(hier.cells * cpu_s / len(tg[0]), 1),
            "sample": f"{len(tg[0])} sampled target cells of the workload, stratified by patch "
                      f"(25% within 2 cells of a level interface), each summed over every "
                      f"active source cell; {cpu_s:.1f} s"}
    return tg, ox, oy, info


# ---------------------------------------------------------------------------
# batch-64: 64 independent hierarchies per step
# ---------------------------------------------------------------------------

def batch_setup(td, torch, synth, ctx, dtype, slopes, count=64):
    """The 64-disk batch as benched (seed 4): plans, device fields, outputs
    and the td_batch.  Returns (disks, host_fields, plans, fields, batch,
    outs)."""
    disks = synth.config4(seed=4, count=count)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    plans, fields, hosts = [], [], []
    for hier, fn in disks:
        plans.append(ctx.plan(hier, dtype))
        h = host_fields(synth, hier, fn, slopes)
        hosts.append(h)
        fields.append(dev_fields(torch, tdt, h, slopes))
    batch = td.Batch(ctx, plans)
    outs = [p.outputs() for p in plans]
    return disks, hosts, plans, fields, batch, outs


def run_batch(args, td, torch, synth):
    """64 independent hierarchies per step, one batched launch set."""
    import numpy as np
    ctx = td.Context(0)
    if args.tune:
        ctx.autotune(args.dtype, 1024, args.tune)
    disks, hosts, plans, fields, batch, outs = batch_setup(td, torch, synth, ctx, args.dtype,
                                                          args.slopes)
    use_graph = args.mode == "graph"
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.solve(fields, outs, use_graph=use_graph, stream=stream)
    torch.cuda.synchronize()
    ctx.timing(True, passes=["col"])
    ctx.timing_read()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            batch.solve(fields, outs, use_graph=use_graph, stream=stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    ctx.timing(False)
    cells = sum(p.cells for p in plans)
    # roofline of the column pass over the batch: one timed eager pass set
    # (graph replays are not timed per pass)
    batch.solve(fields, outs, use_graph=False, stream=stream)
    ctx.timing(True, passes=["col"])
    ctx.timing_read()
    reps = 5
    for _ in range(reps):
        batch.solve(fields, outs, use_graph=False, stream=stream)
    torch.cuda.synchronize()
    ms, launches = ctx.timing_read()["col"]
    ctx.timing(False)
    col_bytes = sum(p.traffic(args.slopes)["col"] for p in plans)
    col_s = ms / 1000.0 / reps
    roof = {"bound": "hbm", "kernel": "col", "achieved": round(col_bytes / col_s / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(col_bytes / col_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_us_per_batch": round(col_s * 1e6, 2), "launches_per_batch": launches / reps,
            "alg_bytes_per_batch": int(col_bytes)}
    cpu = None
    if not args.no_cpu:
        import oracle
        # 8 stratified targets per member, every member summed over all its
        # active sources, about args.cpu_seconds in all
        tgs, gxs, gys, oxs, oys = [], [], [], [], []
        t0 = time.perf_counter()
        ntg = 0
        for k, ((hier, _), h) in enumerate(zip(disks, hosts)):
            tg = synth.sample_targets(hier, 8, seed=40 + k)
            sig, dx, dy = h
            if args.slopes == "estimate":
                dx, dy = oracle.slopes(hier, sig)
            ox, oy = oracle.forces(hier, sig, dx, dy, tg, nthreads=oracle_threads())
            gxs.append(sampled_values(outs[k][0], tg))
            gys.append(sampled_values(outs[k][1], tg))
            oxs.append(ox)
            oys.append(oy)
            ntg += len(tg[0])
        cpu_s = time.perf_counter() - t0
        gx, gy, ox, oy = (np.concatenate(a) for a in (gxs, gys, oxs, oys))
        err = math.sqrt((((gx - ox) ** 2).sum() + ((gy - oy) ** 2).sum()) /
                        ((ox ** 2).sum() + (oy ** 2).sum()))
        cpu = {"value": round(ntg / cpu_s, 2), "unit": "cells/s", "cores": oracle_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{ntg} sampled target cells, 8 per member hierarchy, each summed "
                         f"over every active source cell of its hierarchy; {cpu_s:.1f} s",
               "rel_l2_vs_oracle_sampled": err}
    batch.close()
    return {
        "metric": METRIC,
        "value": cells * args.steps / el, "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "batch-64", "hierarchies": len(plans), "cells_per_step": cells,
                   "mode": args.mode, "slopes": args.slopes,
                   "workspace_bytes": batch_ws_bytes(plans),
                   "python_gc": "paused in timed loops"},
        "roofline": roof, "cpu_baseline": cpu,
    }


def batch_ws_bytes(plans):
    return int(sum(p.footprint()[0] for p in plans))


# ---------------------------------------------------------------------------
# serving: Poisson arrivals of mixed hierarchies
# ---------------------------------------------------------------------------

def serve_block(args, td, torch, synth):
    """Poisson arrivals (mean rate args.rate, seed 5) of mixed hierarchies
    (base N in {128..1024}, 1-5 levels) into the serving loop.  Request types
    are drawn from the arrivals themselves: args.types hierarchies are
    planned before the run; a fraction args.unseen of the arrivals carry a
    hierarchy of their own that no plan exists for, which the server plans
    while other flights run.  Returns the serving record."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(5))
    reqs = synth.config5_requests(seed=5, rate=args.rate, duration=args.duration)
    ctx = td.Context(0, hbm_budget=int(args.budget_gb * (1 << 30)))
    if args.tune:
        ctx.autotune(args.dtype, 2048, args.tune)
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    ntypes = args.types
    types = []
    tp = time.perf_counter()
    for k in range(ntypes):
        _, hier, (order, alpha, fseed) = reqs[k % len(reqs)]
        fn = synth.request_sigma(order, alpha, fseed, hier.h0)
        plan = ctx.plan(hier, args.dtype)
        outs = [plan.outputs() for _ in range(2)]
        types.append((plan, dev_fields(torch, tdt, host_fields(synth, hier, fn, args.slopes),
                                       args.slopes), outs))
    plan_s = time.perf_counter() - tp
    log(f"serve: planned {ntypes} request types in {plan_s:.1f} s")
    srv = td.Server(ctx, max_inflight=args.inflight, max_batch=args.max_batch)
    srv.set_queue_limit(args.queue_limit)
    for plan, f, outs in types:
        srv.submit(plan, *f[:3], *outs[0], slopes=f[3])
    srv.drain()
    torch.cuda.synchronize()
    st0 = srv.stats()
    arrivals = [t for t, _, _ in reqs]
    pick = rng.integers(0, ntypes, len(arrivals))
    unseen = rng.random(len(arrivals)) < args.unseen
    # unseen arrivals keep their own hierarchy (no plan exists for it); their
    # input and output buffers depend only on the patch sides, so they reuse
    # those of a planned type of the same shape (every level of a request
    # has N^2 cells), or of a shape prepared here, before the run
    shape_bufs = {}
    for plan, f, outs in types:
        shape_bufs.setdefault(tuple(plan.sizes), (f, outs))
    fresh = {}
    for k in np.nonzero(unseen)[0]:
        _, hier, _ = reqs[k]
        shp = tuple(p.n for p in hier.patches)
        if shp not in shape_bufs:
            fn = synth.disk_dn(3, 0.8)
            f = dev_fields(torch, tdt, host_fields(synth, hier, fn, args.slopes), args.slopes)
            outs = [tuple([torch.empty((n, n), dtype=tdt, device="cuda") for n in shp]
                          for _ in range(2)) for _ in range(2)]
            shape_bufs[shp] = (f, outs)
        fresh[int(k)] = (hier, shp)
    tickets = []
    refused = 0
    t0 = time.perf_counter()
    next_log = 1.0
    for k, ta in enumerate(arrivals):
        while time.perf_counter() - t0 < ta:
            pass
        try:
            if k in fresh:
                hier, shp = fresh[k]
                f, outs = shape_bufs[shp]
                tk, _, _ = srv.submit_hierarchy(hier, args.dtype, *f[:3], *outs[k % 2],
                                                queue_if_full=False, slopes=f[3])
                tickets.append((tk, hier.cells, True))
            else:
                plan, f, outs = types[pick[k]]
                tk, _, _ = srv.submit(plan, *f[:3], *outs[k % 2], queue_if_full=False,
                                      slopes=f[3])
                tickets.append((tk, plan.cells, False))
        except td.TdError as e:
            if e.status != 6:  # TD_EBUSY: the bounded queue is full
                raise
            refused += 1
        if ta >= next_log:
            log(f"serve t={ta:.1f} s: {len(tickets)} admitted, {refused} refused, "
                f"{srv.stats()['completed'] - st0['completed']} completed")
            next_log += 1.0
    t_arr = time.perf_counter() - t0
    srv.drain()
    el = time.perf_counter() - t0
    lats, lats_new = [], []
    cells = 0
    for tk, c, new in tickets:
        done, lat = srv.poll(tk)
        assert done
        (lats_new if new else lats).append(lat)
        cells += c
    st = srv.stats()
    st = {k: st[k] - st0[k] if k != "peak_queue" else st[k] for k in st}
    all_l = np.array(lats + lats_new)
    srv.close()
    for plan, _, _ in types:
        plan.close()
    ctx.close()
    rec = {"workload": "serve", "offered_rate": args.rate, "duration_s": args.duration,
           "offered": len(arrivals), "admitted": len(tickets), "refused": refused,
           "unseen_hierarchies": int(sum(1 for _, _, n in tickets if n)),
           "unseen_frac_of_arrivals": round(float(unseen.mean()), 3),
           "arrival_window_s": round(t_arr, 3), "wall_s": round(el, 3),
           "sustained_req_per_s": round(len(tickets) / el, 1),
           "cells_per_s": cells / el,
           "p50_ms": float(np.percentile(all_l, 50) * 1e3),
           "p99_ms": float(np.percentile(all_l, 99) * 1e3),
           "mean_ms": float(all_l.mean() * 1e3),
           "p50_ms_unseen": float(np.percentile(lats_new, 50) * 1e3) if lats_new else None,
           "request_types_planned_before": ntypes, "plan_types_s": round(plan_s, 2),
           "max_inflight": args.inflight, "max_batch": args.max_batch,
           "queue_limit": args.queue_limit, "hbm_budget_gb": args.budget_gb,
           "slopes": args.slopes, **st}
    return rec


def run_serve(args, td, torch, synth):
    s = serve_block(args, td, torch, synth)
    return {
        "metric": METRIC,
        "value": s["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": s["admitted"],
        "warmup": args.types, "ms_per_step": 1000 * s["wall_s"] / max(1, s["admitted"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic", "config": {"workload": "serve", "offered_rate": args.rate},
        "serving": s, "roofline": None, "cpu_baseline": None,
    }


# ---------------------------------------------------------------------------
# one hierarchy per step
# ---------------------------------------------------------------------------

def timed_solves(step, steps, warmup, ctx, timed_passes):
    """Warm-up, then `steps` solves between two synchronisations; the passes
    in `timed_passes` are timed with HIP events on the solve stream over the
    measured region.  Returns (seconds, {pass: (ms, launches)})."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if timed_passes:
        ctx.timing(True, passes=timed_passes)
        ctx.timing_read()
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    passes = ctx.timing_read() if timed_passes else None
    ctx.timing(False)
    return el, passes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--mode", default="eager", choices=["eager", "graph"])
    ap.add_argument("--quantity", default="force", choices=["force", "potential"],
                    help="force (the metric) or the potential (a TD_POTENTIAL plan)")
    ap.add_argument("--slopes", default="given", choices=["estimate", "given"],
                    help="given: central differences of the analytic sigma passed in (the "
                         "default); estimate: sigma in, slopes from it inside the solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving block")
    ap.add_argument("--no-estimate-leg", action="store_true",
                    help="skip the timing with the slopes estimated in the solve")
    ap.add_argument("--tune", metavar="DB", default=None,
                    help="autotune launch shapes first (JSON-lines database path)")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: mean arrivals per s")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals")
    ap.add_argument("--queue-limit", type=int, default=256,
                    help="serve: requests waiting for admission at most (others refused)")
    ap.add_argument("--types", type=int, default=48,
                    help="serve: hierarchies planned before the run")
    ap.add_argument("--unseen", type=float, default=0.1,
                    help="serve: fraction of arrivals with a hierarchy planned during the run")
    ap.add_argument("--inflight", type=int, default=4, help="serve: concurrent batches")
    ap.add_argument("--max-batch", type=int, default=16, help="serve: requests per batch")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: HBM budget (GiB)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run plain copies of this many MiB first (counter calibration)")
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
    log(f"{args.workload}: plan built in {plan_s:.3f} s")

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
    if args.mode == "eager" and args.warmup > n_first:
        warm = ctx.timing_read()
    ctx.timing(False)
    dom = max(warm, key=lambda p: warm[p][0]) if warm else None
    elapsed, passes = timed_solves(step, args.steps, 0, ctx, [dom] if dom else None)
    ms_per_step = 1000.0 * elapsed / args.steps
    value = cells * args.steps / elapsed
    log(f"{args.workload} {args.dtype}: {ms_per_step:.4f} ms per solve, {value:.4e} cells/s")

    # latency of one solve on an idle device: enqueue to completion, each
    # solve synchronised (after the timed region, so it does not change it)
    lat = []
    with gc_paused():
        for _ in range(max(50, min(200, args.steps))):
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
    lat = np.array(lat) * 1e3
    latency = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "samples": len(lat),
               "how": "single solves, each from enqueue to completion (host clock), device idle"}

    # roofline of the dominant pass (algorithmic bytes / mean launch time,
    # HIP events on the solve stream)
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

    # the same workload with sigma in and the slopes estimated in the solve
    est = None
    if not args.no_estimate_leg and args.slopes == "given" and args.mode == "eager":
        Se = dev_fields(torch, tdt, (sig, None, None), "estimate")[0]
        step_e = lambda: plan.solve(Se, None, None, FX, FY, stream=stream, slopes="estimate")
        el_e, _ = timed_solves(step_e, args.steps, 3, ctx, None)
        est = {"value": cells * args.steps / el_e, "unit": "cells/s",
               "ms_per_step": 1000.0 * el_e / args.steps,
               "alg_bytes_per_solve": {k: int(v) for k, v in plan.traffic("estimate").items()}}
        # the timed outputs were overwritten: redo the measured solve
        step()
        torch.cuda.synchronize()

    # CPU baseline: the oracle on a bounded sample of the same workload, and
    # the error of this run's result against it
    cpu = tg = ox = oy = None
    acc = None
    if not args.no_cpu:
        import oracle
        odx, ody = (oracle.slopes(hier, sig) if args.slopes == "estimate" else (dx, dy))
        pot = args.quantity == "potential"
        tg, ox, oy, cpu = oracle_sample(hier, sig, odx, ody, args.cpu_seconds, pot)
        gx = sampled_values(FX, tg)
        gy = np.zeros_like(gx) if pot else sampled_values(FY, tg)
        acc = errors(hier, tg, gx, gy, ox, oy)
        log(f"oracle sample: {cpu['sample']}; rel-L2 {acc['rel_l2']:.3e}")

    # the plain per-solve FP64 GPU path (eager, one solve per call, FP64
    # throughout) on the same workload, for the speed-up of this run over it
    fp64 = None
    if not args.no_fp64_leg and not (args.dtype == "f64" and args.mode == "eager"):
        S64, DX64, DY64, _ = dev_fields(torch, torch.float64, (sig, dx, dy), args.slopes)
        ctx64 = td.Context(0)
        plan64 = ctx64.plan(hier, "f64", quantity=args.quantity)
        FX64, FY64 = plan64.outputs()
        k64 = max(3, args.steps // 4)
        step64 = lambda: plan64.solve(S64, DX64, DY64, FX64, FY64, stream=stream, slopes=SL)
        el64, _ = timed_solves(step64, k64, 3, ctx64, None)
        v64 = cells * k64 / el64
        fp64 = {"value": v64, "unit": "cells/s", "steps": k64,
                "ms_per_step": 1000.0 * el64 / k64, "speedup": value / v64}
        if tg is not None:
            gx = sampled_values(FX64, tg)
            gy = np.zeros_like(gx) if FY64 is None else sampled_values(FY64, tg)
            fp64["vs_oracle_sampled"] = errors(hier, tg, gx, gy, ox, oy)
        plan64.close()
        ctx64.close()
        del S64, DX64, DY64, FX64, FY64

    serving = None
    if not args.no_serve and args.workload == DEFAULT_WORKLOAD:
        plan.close()
        ctx.close()
        torch.cuda.empty_cache()
        serving = serve_block(args, td, torch, synth)
        log(f"serving: {serving['sustained_req_per_s']} req/s sustained, p50 "
            f"{serving['p50_ms']:.2f} ms, p99 {serving['p99_ms']:.2f} ms, "
            f"{serving['refused']} refused")

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
        "vs_oracle_sampled": acc,
        "slopes_estimate": est,
        "fp64_per_solve_gpu": fp64,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
