"""Parity at the benchmarked sizes and precisions, through the C ABI.

* four-level 512^2 (the default benchmark workload) in FP64 (rel-L2 <= 1e-12)
  and FP32 (<= 1e-5) against one oracle run on 1024 stratified targets (25%
  within 2 cells of a level interface), asserted overall and on every level;
* the 64-disk batch exactly as benchmarked (seed 4, FP32, slopes passed in,
  hipGraph replays), 16 stratified targets per member;
* a five-level 1024^2 ratio-2 request (m = 16 between its outer levels)
  served inside a mix of other requests, 256 stratified targets.

The oracle is the plain direct sum of Section 2.1 (eqs. eqndPhi, eqnSigma);
the GPU path evaluates the same sums as the FFT convolutions of Section 2.2
(Cases 1', 2' and 3', eqs. eqnbmnn, eqnbnmn).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import report, sampled, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1603_03142_amd as td
    c = td.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def config3_reference():
    """The default benchmark workload with the slopes of the central-difference
    rule, and the oracle at 1024 stratified targets (one run, shared by the
    FP64 and FP32 checks)."""
    hier, fn = synth.config3()
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    tg = synth.sample_targets(hier, 1024, seed=31)
    print(f"config3: oracle on {len(tg[0])} targets", flush=True)
    ox, oy = oracle.forces(hier, sig, dx, dy, tg)
    return hier, sig, dx, dy, tg, ox, oy


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_config3_stratified(ctx, config3_reference, dtype, tol):
    import torch
    hier, sig, dx, dy, tg, ox, oy = config3_reference
    tdt = torch.float64 if dtype == "f64" else torch.float32
    print(f"config3 {dtype}: solve", flush=True)
    plan = ctx.plan(hier, dtype)
    fx, fy = plan.solve(to_dev(sig, tdt), to_dev(dx, tdt), to_dev(dy, tdt))
    torch.cuda.synchronize()
    gx = [a.double().cpu().numpy() for a in fx]
    gy = [a.double().cpu().numpy() for a in fy]
    sx, sy = sampled(hier, gx, gy, tg)
    err, per, _ = report(f"config3 {dtype}", hier, tg, sx, sy, ox, oy)
    assert len(per) == 4
    assert err <= tol
    for lvl, e in per.items():
        assert e <= tol, (lvl, e)
    # covered cells are written as 0
    for k, p in enumerate(hier.patches):
        cov = synth.covered_mask(hier, p)
        assert np.all(gx[k][cov] == 0) and np.all(gy[k][cov] == 0)
    plan.close()


def test_batch64_as_benched(ctx):
    """The 64-disk batch of the benchmark (bench.batch_setup), replayed from
    its hipGraph, against the oracle on 16 targets per member."""
    import torch
    import bench
    import paper_1603_03142_amd as td
    print("batch-64: plans", flush=True)
    disks, hosts, plans, fields, batch, outs = bench.batch_setup(td, torch, synth, ctx, "f32",
                                                                "given")
    stream = torch.cuda.current_stream()
    for _ in range(3):  # capture, then replays
        batch.solve(fields, outs, use_graph=True, stream=stream)
    torch.cuda.synchronize()
    print("batch-64: oracle", flush=True)
    all_g, all_o = [], []
    worst = 0.0
    for k, ((hier, _), (sig, dx, dy)) in enumerate(zip(disks, hosts)):
        tg = synth.sample_targets(hier, 16, seed=400 + k)
        ox, oy = oracle.forces(hier, sig, dx, dy, tg)
        gx = [a.double().cpu().numpy() for a in outs[k][0]]
        gy = [a.double().cpu().numpy() for a in outs[k][1]]
        sx, sy = sampled(hier, gx, gy, tg)
        num = ((sx - ox) ** 2).sum() + ((sy - oy) ** 2).sum()
        den = (ox ** 2).sum() + (oy ** 2).sum()
        e = float(np.sqrt(num / den))
        worst = max(worst, e)
        assert e <= 1e-5, (k, e, [(p.level, p.n) for p in hier.patches])
        all_g.append((sx, sy))
        all_o.append((ox, oy))
    gx = np.concatenate([a for a, _ in all_g])
    gy = np.concatenate([b for _, b in all_g])
    ox = np.concatenate([a for a, _ in all_o])
    oy = np.concatenate([b for _, b in all_o])
    err = float(np.sqrt((((gx - ox) ** 2).sum() + ((gy - oy) ** 2).sum()) /
                        ((ox ** 2).sum() + (oy ** 2).sum())))
    print(f"batch-64 graph f32: rel-L2 {err:.3e} over {len(gx)} targets, worst member "
          f"{worst:.3e}", flush=True)
    assert err <= 1e-5
    batch.close()


def test_served_five_level_1024(ctx):
    """A five-level 1024^2 ratio-2 request (Case-2 / Case-3 pairs up to
    m = 16) served among other requests; its result against the oracle on
    256 stratified targets, overall and per level."""
    import torch
    import paper_1603_03142_amd as td
    rng = np.random.Generator(np.random.PCG64(55))
    big = synth._random_nested(rng, 1024, 5)
    fn = synth.request_sigma(4, 0.8, 12345, big.h0)
    sig, dx, dy = synth.sample_fields(big, fn, "central")
    tdt = torch.float32
    print("served 5x1024: plan", flush=True)
    plan = ctx.plan(big, "f32")
    others = []
    for k, n in enumerate((128, 256, 512, 256, 128, 512)):
        h = synth._random_nested(rng, n, 1 + k % 4)
        f = synth.sample_fields(h, synth.disk_dn(2, 0.7), "central")
        others.append((ctx.plan(h, "f32"), [to_dev(a, tdt) for a in f]))
    srv = td.Server(ctx, max_inflight=3, max_batch=4)
    tickets = []
    for k, (p, f) in enumerate(others[:3]):
        tickets.append(srv.submit(p, *f)[0])
    t_big, fx, fy = srv.submit(plan, to_dev(sig, tdt), to_dev(dx, tdt), to_dev(dy, tdt))
    for p, f in others[3:]:
        tickets.append(srv.submit(p, *f)[0])
    srv.drain()
    done, _ = srv.poll(t_big)
    assert done
    for t in tickets:
        assert srv.poll(t)[0]
    torch.cuda.synchronize()
    tg = synth.sample_targets(big, 256, seed=56)
    print(f"served 5x1024: oracle on {len(tg[0])} targets", flush=True)
    ox, oy = oracle.forces(big, sig, dx, dy, tg)
    gx = [a.double().cpu().numpy() for a in fx]
    gy = [a.double().cpu().numpy() for a in fy]
    sx, sy = sampled(big, gx, gy, tg)
    err, per, _ = report("served five-level 1024^2 f32", big, tg, sx, sy, ox, oy)
    assert len(per) == 5
    assert err <= 1e-5
    for lvl, e in per.items():
        assert e <= 1e-5, (lvl, e)
    srv.close()
