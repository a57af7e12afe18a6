"""Batches, graph replays, the serving loop, full-size workloads and the
largest size, through the C ABI.

Batch and graph solves run the same jobs as single solves and must agree
bit for bit; served results must agree with solo results within the FP32
tolerance (they agree bit for bit as well, since a request's jobs do not
depend on its neighbours).  Full-size parity is checked on sampled targets
against the oracle.
"""
import math
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import gpu_solve, rand_fields, rel_l2, rel_l2_full, sampled, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1603_03142_amd as td
    c = td.Context(0)
    yield c
    c.close()


def _mix(seed=21, count=6, sizes=(24, 40, 64)):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.choice(sizes))
        lv = [(n, 0, 0)]
        for _ in range(int(rng.integers(0, 3))):
            pn, pox, poy = lv[-1]
            w = int(rng.integers(2, pn // 2 + 1))
            kx, ky = (int(v) for v in rng.integers(0, pn - w + 1, 2))
            lv.append((2 * w, 2 * (pox + kx), 2 * (poy + ky)))
        out.append(synth.nested_hierarchy(-1.0, -1.0, 2.0 / n, 2, lv))
    return out


def _dev_fields(hier, seed, dtype):
    import torch
    td_ = torch.float32 if dtype == "f32" else torch.float64
    s, x, y = rand_fields(hier, seed)
    return (to_dev(s, td_), to_dev(x, td_), to_dev(y, td_)), (s, x, y)


def _host(outs):
    """[(fx list, fy list)] of tensors -> the same structure of numpy arrays."""
    return [tuple([t.double().cpu().numpy() for t in lst] if lst is not None else [] for lst in pair)
            for pair in outs]


@pytest.mark.parametrize("launch", ["persistent", "direct"])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_solves(ctx, use_graph, launch):
    import torch
    import paper_1603_03142_amd as td
    hiers = _mix()
    plans = [ctx.plan(h, "f32") for h in hiers]
    fields = [_dev_fields(h, 100 + k, "f32")[0] for k, h in enumerate(hiers)]
    # every other member estimates its slopes from sigma (tagged slots in the
    # batch's device pointer table)
    fields = [f if k % 2 == 0 else (f[0], None, None, "estimate") for k, f in enumerate(fields)]
    single = []
    for p, f in zip(plans, fields):
        fx, fy = p.solve(*f[:3], slopes=f[3] if len(f) > 3 else "given")
        single.append((fx, fy))
    torch.cuda.synchronize()
    batch = td.Batch(ctx, plans)
    batch.set_launch(launch)
    res = batch.solve(fields, use_graph=use_graph)
    torch.cuda.synchronize()
    for (ax, ay), (bx, by) in zip(_host(single), _host(res)):
        for a, b in zip(ax + ay, bx + by):
            assert np.array_equal(a, b)
    batch.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_persistent_launches_equal_direct(ctx, dtype):
    """Deep hierarchies of several lengths in one batch (in FP64 with two
    potential plans among the force plans): the persistent column launches
    (work lists per XCD, stealing, counters zeroed by a kernel ahead of each
    solve) give the direct launches' results bit for bit, eagerly and on
    every graph replay, with the launch mode switched between."""
    import torch
    import paper_1603_03142_amd as td
    rng = np.random.Generator(np.random.PCG64(808))
    hiers = [synth._random_nested(rng, n, lv) for n, lv in
             ((256, 3), (128, 4), (512, 2), (64, 1), (256, 2), (128, 3), (64, 2), (256, 4))]
    quantity = ["force"] * len(hiers)
    if dtype == "f64":
        quantity[1] = quantity[4] = "potential"
    plans = [ctx.plan(h, dtype, quantity=q) for h, q in zip(hiers, quantity)]
    fields = [_dev_fields(h, 300 + k, dtype)[0] for k, h in enumerate(hiers)]
    batch = td.Batch(ctx, plans)
    batch.set_launch("direct")
    want = _host(batch.solve(fields))
    torch.cuda.synchronize()
    batch.set_launch("persistent")
    outs = [p.outputs() for p in plans]
    for rep, graph in enumerate((False, False, True, True, True)):
        print(f"persistent batch: solve {rep} graph={graph}", flush=True)
        batch.solve(fields, outs=outs, use_graph=graph)
        torch.cuda.synchronize()
        for k, ((ax, ay), (bx, by)) in enumerate(zip(want, _host(outs))):
            for a, b in zip(ax + ay, bx + by):
                assert np.array_equal(a, b), f"solve {rep} member {k}"
        for o in outs:
            for t in o[0] + (o[1] or []):
                t.fill_(float("nan"))
    batch.set_launch("direct")
    again = _host(batch.solve(fields, use_graph=True))
    torch.cuda.synchronize()
    for (ax, ay), (bx, by) in zip(want, again):
        for a, b in zip(ax + ay, bx + by):
            assert np.array_equal(a, b)
    batch.close()


def test_graph_replays_track_inputs(ctx):
    """A captured batch replayed several times, with other GPU work and new
    inputs between replays, matches an eager solve of every replay's inputs."""
    import torch
    import paper_1603_03142_amd as td
    hiers = _mix(seed=7, count=3)
    plans = [ctx.plan(h, "f32") for h in hiers]
    batch = td.Batch(ctx, plans)
    outs = [p.outputs() for p in plans]
    for rep in range(4):
        fields = [_dev_fields(h, 1000 * rep + k, "f32")[0] for k, h in enumerate(hiers)]
        batch.solve(fields, outs=outs, use_graph=True)
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()  # unrelated eager work between replays
        torch.cuda.synchronize()
        got = _host(outs)
        for k, (p, f) in enumerate(zip(plans, fields)):
            fx, fy = p.solve(*f)
            torch.cuda.synchronize()
            want = _host([(fx, fy)])[0]
            for a, b in zip(got[k][0] + got[k][1], want[0] + want[1]):
                assert np.array_equal(a, b), f"replay {rep} member {k}"
    batch.close()


def test_server_alone_equals_in_mix(ctx):
    import torch
    import paper_1603_03142_amd as td
    hiers = _mix(seed=3, count=12)
    plans = [ctx.plan(h, "f32") for h in hiers]
    fields = [_dev_fields(h, 300 + k, "f32")[0] for k, h in enumerate(hiers)]
    srv = td.Server(ctx, max_inflight=3, max_batch=8)
    # alone
    t, fx, fy = srv.submit(plans[0], *fields[0])
    srv.drain()
    done, lat = srv.poll(t)
    assert done and lat > 0
    alone = _host([(fx, fy)])[0]
    # in a mix: the same request among the others, several times over
    tickets = []
    for rep in range(3):
        for k in range(len(plans)):
            tickets.append((k, *srv.submit(plans[k], *fields[k])))
    srv.drain()
    lats = []
    for k, tk, fx, fy in tickets:
        done, lat = srv.poll(tk)
        assert done
        lats.append(lat)
        if k == 0:
            mix = _host([(fx, fy)])[0]
            num = sum(((a - b) ** 2).sum() for a, b in zip(mix[0] + mix[1], alone[0] + alone[1]))
            den = sum((b ** 2).sum() for b in alone[0] + alone[1])
            assert math.sqrt(num / den) <= 1e-5
    st = srv.stats()
    assert st["completed"] == 1 + 3 * len(plans)
    assert st["batches"] >= 2
    srv.close()


def test_server_mixed_quantities_and_slopes(ctx):
    """Force and potential plans, given and estimated slopes, interleaved in
    one server: every request's output equals its own single solve bit for
    bit (a flight runs the batch launches, which compute each member exactly
    as a single solve does)."""
    import torch
    import paper_1603_03142_amd as td
    hiers = _mix(seed=11, count=8)
    cases = []
    for k, h in enumerate(hiers):
        quantity = "potential" if k % 3 == 1 else "force"
        slopes = "estimate" if k % 2 else "given"
        plan = ctx.plan(h, "f32", quantity=quantity)
        f = _dev_fields(h, 500 + k, "f32")[0]
        f = f if slopes == "given" else (f[0], None, None)
        cases.append((plan, f, slopes))
    single = []
    for plan, f, slopes in cases:
        single.append(plan.solve(*f, slopes=slopes))
    torch.cuda.synchronize()
    srv = td.Server(ctx, max_inflight=2, max_batch=5)
    tickets = []
    for rep in range(2):
        for k, (plan, f, slopes) in enumerate(cases):
            tickets.append((k, *srv.submit(plan, *f, slopes=slopes)))
    srv.drain()
    for k, tk, fx, fy in tickets:
        done, _ = srv.poll(tk)
        assert done
        want_x, want_y = single[k]
        for a, b in zip(fx, want_x):
            assert torch.equal(a, b), k
        if cases[k][0].quantity == "potential":
            assert fy is None
        else:
            for a, b in zip(fy, want_y):
                assert torch.equal(a, b), k
    assert srv.stats()["completed"] == 2 * len(cases)
    srv.close()


def test_server_cancel_and_budget(ctx):
    import paper_1603_03142_amd as td
    hier = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 128, 2, [(128, 0, 0), (128, 64, 64)])
    plan = ctx.plan(hier, "f32")
    f = _dev_fields(hier, 5, "f32")[0]
    srv = td.Server(ctx, max_inflight=1, max_batch=1)
    tickets = [srv.submit(plan, *f)[0] for _ in range(6)]
    cancelled = 0
    try:
        srv.cancel(tickets[-1])
        cancelled = 1
    except td.TdError as e:       # already started: allowed, reported as EINVAL
        assert e.status == 1
    srv.drain()
    st = srv.stats()
    assert st["cancelled"] == cancelled
    assert st["completed"] == 6 - cancelled
    srv.close()
    # a context whose budget cannot hold a request's workspace refuses it
    small = td.Context(0, hbm_budget=1 << 20)
    with pytest.raises(td.TdError) as ei:
        small.plan(synth.nested_hierarchy(-1.0, -1.0, 2.0 / 256, 2, [(256, 0, 0)]), "f32")
    assert ei.value.status == 4  # TD_ENOMEM
    small.close()


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_config2_sampled(ctx, dtype, tol):
    """Two nested 256^2 levels, Maclaurin + clump: 256 sampled targets."""
    hier, fn = synth.config2()
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    gx, gy = gpu_solve(ctx, hier, sig, dx, dy, dtype)
    tg = synth.sample_targets(hier, 256, seed=11)
    ox, oy = oracle.forces(hier, sig, dx, dy, tg)
    sx, sy = sampled(hier, gx, gy, tg)
    err = rel_l2(sx, sy, ox, oy)
    print(f"config2 {dtype} sampled rel-L2 {err:.3e}")
    assert err <= tol


def test_config3_sampled_f32(ctx):
    """Four nested 512^2 levels snapped near (0.3, 0), D2 disk x lognormal:
    sampled targets, FP32 FFTs with FP64-built spectra."""
    hier, fn = synth.config3()
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    gx, gy = gpu_solve(ctx, hier, sig, dx, dy, "f32")
    tg = synth.sample_targets(hier, 48, seed=12)
    ox, oy = oracle.forces(hier, sig, dx, dy, tg)
    sx, sy = sampled(hier, gx, gy, tg)
    err = rel_l2(sx, sy, ox, oy)
    print(f"config3 f32 sampled rel-L2 {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("workload,count,dtype,tol", [
    ("two-level-256", 256, "f32", 1e-5), ("two-level-256", 128, "f64", 1e-12),
    ("four-level-512", 48, "f32", 1e-5), ("example1-1024", 32, "f32", 1e-5)])
def test_bench_configuration_sampled(ctx, workload, count, dtype, tol):
    """The configurations bench.py times, as it times them: sigma in, the
    slopes estimated inside the solve; oracle on sampled targets with the
    oracle's own slope estimate of the same sigma."""
    import bench
    hier, fn = bench.workload(workload)
    sig, _, _ = synth.sample_fields(hier, fn, "none")
    gx, gy = gpu_solve(ctx, hier, sig, None, None, dtype, slopes="estimate")
    tg = synth.sample_targets(hier, count, seed=17)
    ox, oy = oracle.forces(hier, sig, *oracle.slopes(hier, sig), tg)
    sx, sy = sampled(hier, gx, gy, tg)
    err = rel_l2(sx, sy, ox, oy)
    print(f"{workload} {dtype} estimated slopes, sampled rel-L2 {err:.3e}")
    assert err <= tol


def test_fp32_vs_fp64_full_field(ctx):
    hier, fn = synth.config2()
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    ax, ay = gpu_solve(ctx, hier, sig, dx, dy, "f64")
    bx, by = gpu_solve(ctx, hier, sig, dx, dy, "f32")
    err = rel_l2_full(hier, bx, by, ax, ay)
    print(f"config2 f32 vs f64 rel-L2 {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_largest_level(ctx, dtype):
    """One 2048^2 level (transform length 4096, the largest; in FP64 the
    passes hold 136 KiB of LDS per workgroup): sampled targets."""
    n = 2048
    hier = synth.nested_hierarchy(-1.0, -1.0, 2.0 / n, 2, [(n, 0, 0)])
    fn = synth.disk_dn(2, 0.9)
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    gx, gy = gpu_solve(ctx, hier, sig, dx, dy, dtype)
    tg = synth.sample_targets(hier, 12, seed=13)
    ox, oy = oracle.forces(hier, sig, dx, dy, tg)
    sx, sy = sampled(hier, gx, gy, tg)
    assert rel_l2(sx, sy, ox, oy) <= {"f32": 1e-5, "f64": 1e-12}[dtype]


def test_autotuned_plans_keep_parity(tmp_path):
    import paper_1603_03142_amd as td
    c = td.Context(0)
    db = str(tmp_path / "tune.jsonl")
    c.autotune("f64", 128, db)
    assert open(db).read().count('"pass"') >= 3
    hier = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 40, 2, [(40, 0, 0), (32, 20, 12)])
    sig, dx, dy = rand_fields(hier, 9)
    ox, oy = oracle.forces(hier, sig, dx, dy)
    gx, gy = gpu_solve(c, hier, sig, dx, dy, "f64")
    assert rel_l2_full(hier, gx, gy, ox, oy) <= 1e-12
    c2 = td.Context(0)
    c2.autotune("f64", 128, db)  # read back from the database
    gx2, gy2 = gpu_solve(c2, hier, sig, dx, dy, "f64")
    assert all(np.array_equal(a, b) for a, b in zip(gx + gy, gx2 + gy2))
    c.close()
    c2.close()


def test_timing_and_traffic(ctx):
    import torch
    hier, fn = synth.config1()
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    plan = ctx.plan(hier, "f32")
    f = (to_dev(sig, torch.float32), to_dev(dx, torch.float32), to_dev(dy, torch.float32))
    ctx.timing(True)
    ctx.timing_read()
    for _ in range(3):
        plan.solve(*f)
    torch.cuda.synchronize()
    t = ctx.timing_read()
    ctx.timing(False)
    for p in ("row_fwd", "col", "row_inv"):
        assert t[p][1] == 3 and t[p][0] > 0
    tr = plan.traffic()
    assert all(tr[p] > 0 for p in ("row_fwd", "col", "row_inv"))
    # estimated slopes read sigma only: less in the row pass, the rest equal
    te = plan.traffic("estimate")
    assert te["row_fwd"] < tr["row_fwd"]
    assert all(te[p] == tr[p] for p in ("col", "row_inv", "row_inv_acc"))
    ws, spec = plan.footprint()
    assert ws > 0 and spec > 0


def test_server_queue_limit_refuses(ctx):
    """With the admission queue bounded, submissions beyond it are refused
    (TD_EBUSY) and counted; every admitted one completes."""
    import paper_1603_03142_amd as td
    hier, _ = synth.config3()  # about a millisecond per solve
    plan = ctx.plan(hier, "f32")
    f = _dev_fields(hier, 6, "f32")[0]
    srv = td.Server(ctx, max_inflight=1, max_batch=1)
    srv.set_queue_limit(2)
    ok = busy = 0
    for _ in range(40):
        try:
            srv.submit(plan, *f, queue_if_full=False)
            ok += 1
        except td.TdError as e:
            assert e.status == 6  # TD_EBUSY
            busy += 1
    srv.drain()
    st = srv.stats()
    assert busy > 0 and ok >= 2
    assert st["completed"] == ok and st["refused"] == busy
    srv.close()


def test_server_plans_unseen_hierarchies(ctx):
    """Requests submitted with a hierarchy and no plan: the server plans each
    distinct hierarchy once (off its launch thread) while other requests run,
    and every result equals a single solve of its own plan bit for bit."""
    import torch
    import paper_1603_03142_amd as td
    hiers = _mix(seed=41, count=5)
    fields = [_dev_fields(h, 700 + k, "f32")[0] for k, h in enumerate(hiers)]
    known = ctx.plan(hiers[0], "f32")
    srv = td.Server(ctx, max_inflight=2, max_batch=4)
    tickets = []
    for rep in range(2):
        for k, (h, f) in enumerate(zip(hiers, fields)):
            if k == 0:
                tickets.append((k, *srv.submit(known, *f)))
            else:
                tickets.append((k, *srv.submit_hierarchy(h, "f32", *f)))
    srv.drain()
    st = srv.stats()
    assert st["planned"] == 2 * (len(hiers) - 1) and st["failed"] == 0
    assert st["completed"] == len(tickets)
    for k, tk, fx, fy in tickets:
        done, lat = srv.poll(tk)
        assert done and lat > 0
        p = ctx.plan(hiers[k], "f32")
        wx, wy = p.solve(*fields[k])
        torch.cuda.synchronize()
        for a, b in zip(fx + fy, wx + wy):
            assert torch.equal(a, b), k
        p.close()
    # a polled ticket is forgotten
    with pytest.raises(td.TdError) as ei:
        srv.poll(tickets[0][1])
    assert ei.value.status == 1
    srv.close()


def test_server_waits_for_the_submitting_stream(ctx):
    """Inputs written on the caller's stream right before submission (behind
    a long kernel there) are the ones the flight reads."""
    import torch
    import paper_1603_03142_amd as td
    hier = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 128, 2, [(128, 0, 0), (128, 64, 64)])
    plan = ctx.plan(hier, "f32")
    (s, x, y), _ = _dev_fields(hier, 77, "f32")
    want = plan.solve(s, x, y)
    torch.cuda.synchronize()
    srv = td.Server(ctx, max_inflight=2, max_batch=2)
    side = torch.cuda.Stream()
    s2 = [torch.zeros_like(a) for a in s]
    with torch.cuda.stream(side):
        m = torch.randn(2048, 2048, device="cuda")
        for _ in range(20):
            m = m @ m
            m = m / m.norm()
        for a, b in zip(s2, s):
            a.copy_(b)
    t, fx, fy = srv.submit(plan, s2, x, y, stream=side)
    srv.drain()
    assert srv.poll(t)[0]
    torch.cuda.synchronize()
    for a, b in zip(fx + fy, want[0] + want[1]):
        assert torch.equal(a, b)
    srv.close()


def test_server_budget_admits_workspace_not_pointer_table():
    """A budget that holds a request's workspace but not the flight's device
    pointer table: the request fails with TD_ENOMEM, is never reported done,
    and the server stays usable."""
    import torch
    import paper_1603_03142_amd as td
    hier = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 64, 2, [(64, 0, 0), (64, 32, 32)])
    probe = td.Context(0)
    p = probe.plan(hier, "f32")
    used, _ = probe.usage()
    p.close()
    probe.close()
    ws = td.check_plan(hier, "f32")
    # the plan's own allocations, its workspace (256-byte rounded), and less
    # than the 1024-entry pointer table of a flight
    budget = used + ((ws + 255) & ~255) + 4096
    c = td.Context(0, hbm_budget=budget)
    plan = c.plan(hier, "f32")
    (s, x, y), _ = _dev_fields(hier, 3, "f32")
    srv = td.Server(c, max_inflight=1, max_batch=1)
    tk = srv.submit(plan, s, x, y)[0]
    srv.drain()
    with pytest.raises(td.TdError) as ei:
        srv.poll(tk)
    assert ei.value.status == 4  # TD_ENOMEM
    st = srv.stats()
    assert st["completed"] == 0 and st["failed"] == 1
    srv.close()
    plan.close()
    c.close()
    torch.cuda.synchronize()
