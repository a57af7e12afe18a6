#!/usr/bin/env python3
"""Throughput of the thin-disk force solve on one MI355X.

One step = one full force solve (every pass of the hot path) of the workload:
  two nested levels of 256 x 256 cells, ratio 2, the fine level covering the
  central [-1/2,1/2]^2 of the [-1,1]^2 base; sigma = Maclaurin disk R = 0.8
  plus a Gaussian clump (amplitude 5, width 0.03) at (0.2, 0.1); slopes by
  central differences of the analytic sigma; FP32 FFT passes with
  FP64-built kernel spectra.
Inputs are resident in HBM before the timed region; kernel spectra are
resident (plan built beforehand).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]
                  [--workload two-level-256|single-64|four-level-512]
                  [--mode eager|graph] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def workload(name):
    import synth
    if name == "two-level-256":
        hier, fn = synth.config2()
    elif name == "single-64":
        hier, fn = synth.config1()
    elif name == "four-level-512":
        hier, fn = synth.config3()
    else:
        raise SystemExit(f"unknown workload {name}")
    return hier, fn


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="two-level-256")
    ap.add_argument("--mode", default="eager", choices=["eager", "graph"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tune", metavar="DB", default=None,
                    help="autotune launch shapes first (JSON-lines database path)")
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
    hier, fn = workload(args.workload)
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    dev = lambda arrs: [torch.as_tensor(a, dtype=tdt, device="cuda") for a in arrs]
    S, DX, DY = dev(sig), dev(dx), dev(dy)

    ctx = td.Context(0)
    tune_s = None
    if args.tune:
        t0 = time.perf_counter()
        ctx.autotune(args.dtype, max(p.n for p in hier.patches) * 2, args.tune)
        tune_s = round(time.perf_counter() - t0, 2)
    t0 = time.perf_counter()
    plan = ctx.plan(hier, args.dtype)
    plan_s = time.perf_counter() - t0
    FX, FY = plan.outputs()
    cells = plan.cells
    stream = torch.cuda.current_stream()

    if args.mode == "graph":
        batch = td.Batch(ctx, [plan])
        step = lambda: batch.solve([(S, DX, DY)], [(FX, FY)], use_graph=True, stream=stream)
    else:
        step = lambda: plan.solve(S, DX, DY, FX, FY, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(args.mode == "eager")
    ctx.timing_read()  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    passes = ctx.timing_read() if args.mode == "eager" else None
    ctx.timing(False)
    ms_per_step = 1000.0 * elapsed / args.steps
    value = cells * args.steps / elapsed

    # roofline of the dominant pass (algorithmic bytes / mean launch time)
    roof = None
    traffic = plan.traffic()
    if passes:
        dom = max(passes, key=lambda p: passes[p][0])
        ms, launches = passes[dom]
        per_launch_s = ms / 1000.0 / max(launches, 1)
        launches_per_solve = launches / args.steps
        bytes_per_launch = traffic[dom] / max(launches_per_solve, 1e-30)
        achieved = bytes_per_launch / per_launch_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "avg_launch_us": round(per_launch_s * 1e6, 2),
                "alg_bytes_per_launch": int(bytes_per_launch),
                "passes_us_per_solve": {p: round(1000.0 * passes[p][0] / args.steps, 2)
                                        for p in passes}}

    # CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    acc = None
    if not args.no_cpu:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        probe = synth.sample_targets(hier, 8, seed=1)
        tp0 = time.perf_counter()
        oracle.forces(hier, sig, dx, dy, probe, nthreads=nthreads)
        per_target = (time.perf_counter() - tp0) / len(probe[0])
        count = max(8, min(4096, int(args.cpu_seconds / max(per_target, 1e-9))))
        tg = synth.sample_targets(hier, count, seed=2)
        tp0 = time.perf_counter()
        ox, oy = oracle.forces(hier, sig, dx, dy, tg, nthreads=nthreads)
        cpu_s = time.perf_counter() - tp0
        cpu = {"value": round(len(tg[0]) / cpu_s, 2), "unit": "cells/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"{len(tg[0])} sampled target cells of the workload (25% within 2 "
                         f"cells of a level interface), each summed over every active source "
                         f"cell; {cpu_s:.1f} s"}
        fxc = [f.double().cpu().numpy() for f in FX]
        fyc = [f.double().cpu().numpy() for f in FY]
        gx = np.array([fxc[p][j, i] for p, i, j in zip(*tg)])
        gy = np.array([fyc[p][j, i] for p, i, j in zip(*tg)])
        acc = math.sqrt((((gx - ox) ** 2).sum() + ((gy - oy) ** 2).sum()) /
                        ((ox ** 2).sum() + (oy ** 2).sum()))

    out = {
        "metric": "force-solve cells/s at rel-L2 <=1e-5 vs FP64 oracle",
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
        "config": {"workload": args.workload, "levels": len(hier.patches),
                   "cells_per_level": [p.n for p in hier.patches], "ratio": hier.ratio,
                   "cells_per_solve": cells, "mode": args.mode,
                   "plan_build_s": round(plan_s, 3), "autotune_s": tune_s},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rel_l2_vs_oracle_sampled": acc,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
