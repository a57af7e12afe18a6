"""The allocation-free solve (td_solve_noalloc), through the C ABI.

It runs the same kernels and jobs as td_solve on a fixed device array, so
its outputs must equal td_solve's bit for bit: checked on two calls in a
row, the second with a smaller hierarchy (the array keeps the first call's
contents), FP32 and FP64, given and estimated slopes.  A plan whose
workspace exceeds the array is refused with TD_ENOMEM and writes nothing.
"""
import ctypes

import numpy as np
import pytest

import synth
from gpu_helpers import rand_fields, to_dev

pytestmark = pytest.mark.gpu


def _solve(fn, plan, tensors, slopes):
    """One solve through the C entry point `fn` (td_solve or
    td_solve_noalloc) on torch's current stream; returns (fx, fy)."""
    import torch
    from paper_1603_03142_amd import _binding as B
    sig, dx, dy = tensors
    req, fx, fy = plan.request(sig, dx, dy, slopes=slopes)
    st = fn(ctypes.byref(req), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == B.TD_OK, B.lib().td_last_error().decode()
    torch.cuda.synchronize()
    return [a.cpu() for a in fx], [a.cpu() for a in fy]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_equals_solve_twice_second_smaller(dtype):
    import torch
    import paper_1603_03142_amd as td
    from paper_1603_03142_amd import _binding as B
    lib = B.lib()
    ctx = td.Context(0)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    big = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 256, 2, [(256, 0, 0), (256, 64, 128)])
    small = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 48, 2, [(48, 0, 0), (40, 30, 18), (32, 64, 40)])
    for k, (hier, slopes) in enumerate([(big, "given"), (small, "estimate")]):
        plan = ctx.plan(hier, dtype)
        s, x, y = rand_fields(hier, 50 + k)
        dev = (to_dev(s, tdt), to_dev(x, tdt) if slopes == "given" else None,
               to_dev(y, tdt) if slopes == "given" else None)
        want = _solve(lib.td_solve, plan, dev, slopes)
        got = _solve(lib.td_solve_noalloc, plan, dev, slopes)
        for a, b in zip(got[0] + got[1], want[0] + want[1]):
            assert torch.equal(a, b), (dtype, k)
        assert all(np.isfinite(a.numpy()).all() for a in got[0])
        plan.close()
    ctx.close()


def test_noalloc_refuses_a_workspace_beyond_the_array():
    import torch
    import paper_1603_03142_amd as td
    from paper_1603_03142_amd import _binding as B
    lib = B.lib()
    ctx = td.Context(0)
    hier, _ = synth.config3()  # 275 MB of workspace in FP32
    plan = ctx.plan(hier, "f32")
    s, x, y = rand_fields(hier, 7)
    tdt = torch.float32
    req, fx, fy = plan.request(to_dev(s, tdt), to_dev(x, tdt), to_dev(y, tdt))
    for a in fx:
        a.fill_(123.0)
    torch.cuda.synchronize()
    st = lib.td_solve_noalloc(ctypes.byref(req), None)
    assert st == B.TD_ENOMEM
    assert b"exceeds the fixed scratch" in lib.td_last_error()
    torch.cuda.synchronize()
    assert all(bool((a == 123.0).all()) for a in fx)  # nothing enqueued
    plan.close()
    ctx.close()
