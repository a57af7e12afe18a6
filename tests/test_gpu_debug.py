"""Debug mode: the count of non-finite outputs (NaN / Inf) of every solve of
a context, through the C ABI.  A clean solve counts 0; a NaN planted in one
input cell spreads through the transforms to every output of every level
(covered cells stay 0), and single solves, batches and served requests all
count it."""
import pytest

import synth
from gpu_helpers import rand_fields, to_dev

pytestmark = pytest.mark.gpu


def test_nonfinite_count():
    import torch
    import paper_1603_03142_amd as td
    ctx = td.Context(0)
    hier = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 32, 2, [(32, 0, 0), (32, 16, 8)])
    plan = ctx.plan(hier, "f32")
    s, x, y = (to_dev(a, torch.float32) for a in rand_fields(hier, 4))
    assert ctx.nonfinite_count() == 0  # never enabled: nothing counted
    ctx.set_debug(True)
    plan.solve(s, x, y)
    assert ctx.nonfinite_count() == 0
    active = sum(int((~synth.covered_mask(hier, p)).sum()) for p in hier.patches)
    s[1][3, 5] = float("nan")
    plan.solve(s, x, y)
    n_single = ctx.nonfinite_count()
    assert n_single == 2 * active  # Fx and Fy of every active cell
    batch = td.Batch(ctx, [plan, plan])
    batch.solve([(s, x, y), (s, x, y)])
    assert ctx.nonfinite_count() == 2 * n_single
    srv = td.Server(ctx, max_inflight=1, max_batch=2)
    t = srv.submit(plan, s, x, y)[0]
    srv.drain()
    assert srv.poll(t)[0]
    assert ctx.nonfinite_count() == n_single
    srv.close()
    ctx.set_debug(False)
    plan.solve(s, x, y)
    assert ctx.nonfinite_count() == 0
    batch.close()
    plan.close()
    ctx.close()
