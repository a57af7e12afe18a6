"""MI355X-native thin-disk self-gravity on nested grids.

Python face of ``libthindisk.so`` (C ABI in ``include/thindisk.h``).  PyTorch
supplies device memory and streams; every step of a solve runs in the HIP
kernels of ``csrc/``.

    import paper_1603_03142_amd as td
    ctx = td.Context()
    plan = ctx.plan(hierarchy, "f32")
    fx, fy = plan.solve(sigma, dsdx, dsdy)      # lists of (n, n) tensors per level
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

from . import _binding as B
from ._binding import TdError, lib

__all__ = ["Context", "Plan", "Batch", "Server", "TdError", "lib", "version"]

_DT = {"f32": B.TD_F32, "f64": B.TD_F64}
_SLOPES = {"given": B.TD_SLOPES_GIVEN, "estimate": B.TD_SLOPES_ESTIMATE}
_QUANTITY = {"force": B.TD_FORCE, "potential": B.TD_POTENTIAL}


def version() -> str:
    return lib().td_version().decode()


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_fields(plan: "Plan", arrays, name, required=True):
    torch = _torch()
    if arrays is None:
        if required:
            raise ValueError(f"{name} is required")
        return None
    if len(arrays) != plan.npatches:
        raise ValueError(f"{name}: expected {plan.npatches} arrays (one per patch), got {len(arrays)}")
    for l, (t, n) in enumerate(zip(arrays, plan.sizes)):
        if t is None:
            if required:
                raise ValueError(f"{name}[{l}] is None")
            continue
        if not t.is_cuda or t.dtype != plan.torch_dtype or tuple(t.shape) != (n, n) \
                or not t.is_contiguous():
            raise ValueError(f"{name}[{l}] must be a contiguous {plan.torch_dtype} CUDA tensor "
                             f"of shape ({n}, {n})")
    return arrays


class Context:
    """td_context: one device, resident spectra, HBM budget (0 = none)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        B.check(lib().td_context_create(device, hbm_budget, ctypes.byref(h)), "td_context_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            B.check(lib().td_context_destroy(self.handle), "td_context_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def usage(self):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        B.check(lib().td_context_usage(self.handle, ctypes.byref(a), ctypes.byref(b)),
                "td_context_usage")
        return a.value, b.value

    def set_debug(self, nonfinite: bool = True):
        """Debug mode: count NaN / Inf outputs of every solve (see
        nonfinite_count)."""
        B.check(lib().td_context_set_debug(self.handle, B.TD_DEBUG_NONFINITE if nonfinite else 0),
                "td_context_set_debug")

    def nonfinite_count(self) -> int:
        """Non-finite output values counted since the previous call (waits
        for the device)."""
        n = ctypes.c_uint64()
        B.check(lib().td_debug_nonfinite(self.handle, ctypes.byref(n)), "td_debug_nonfinite")
        return n.value

    def plan(self, hier, dtype: str = "f32", quantity: str = "force") -> "Plan":
        """quantity "force" (solves return (fx, fy)) or "potential" (solves
        return (phi, None))."""
        return Plan(self, hier, dtype, quantity)

    def autotune(self, dtype: str = "f32", max_M: int = 2048, db_path: Optional[str] = None):
        B.check(lib().td_autotune(self.handle, _DT[dtype], max_M,
                                  db_path.encode() if db_path else None), "td_autotune")

    PASSES = ("row_fwd", "col", "row_inv", "row_inv_acc")

    def timing(self, enable: bool = True, passes=None):
        """Time every launch kind (or only those named in `passes`)."""
        mask = 0
        if enable:
            mask = (1 << len(self.PASSES)) - 1 if passes is None else \
                sum(1 << self.PASSES.index(p) for p in passes)
        B.check(lib().td_timing_enable(self.handle, mask), "td_timing_enable")

    def timing_read(self):
        """{pass: (milliseconds, launches)} since the previous read."""
        ms = (ctypes.c_double * len(self.PASSES))()
        n = (ctypes.c_int64 * len(self.PASSES))()
        B.check(lib().td_timing_read(self.handle, ms, n), "td_timing_read")
        return {p: (ms[i], n[i]) for i, p in enumerate(self.PASSES)}

    def kernel_table(self, M: int, kind: int, m: int = 1, kx: int = 0, ky: int = 0,
                     quantity: str = "force", aspect: float = 1.0):
        import numpy as np
        out = np.zeros((6, M, M))
        B.check(lib().td_kernel_table(self.handle, _QUANTITY[quantity], float(aspect), M, kind,
                                      m, kx, ky,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                "td_kernel_table")
        return out


def check_hierarchy(hier) -> None:
    h = B.make_hierarchy(hier)
    B.check(lib().td_hierarchy_check(ctypes.byref(h)), "td_hierarchy_check")


def check_plan(hier, dtype: str = "f32") -> int:
    """td_plan_check: host-only job building and bounds proof; returns the
    workspace bytes."""
    h = B.make_hierarchy(hier)
    ws = ctypes.c_size_t()
    B.check(lib().td_plan_check(ctypes.byref(h), _DT[dtype], ctypes.byref(ws)), "td_plan_check")
    return ws.value


class Plan:
    """td_plan for one hierarchy and dtype; field lists are per patch, in the
    hierarchy's patch order."""

    def __init__(self, ctx: Context, hier, dtype: str = "f32", quantity: str = "force"):
        if dtype not in _DT:
            raise ValueError("dtype must be 'f32' or 'f64'")
        if quantity not in _QUANTITY:
            raise ValueError(f"quantity must be one of {sorted(_QUANTITY)}")
        self.ctx = ctx
        self.dtype = dtype
        self.quantity = quantity
        self.hier = hier
        h = B.make_hierarchy(hier)
        self.npatches = h.npatches
        self.sizes = [h.patches[k].n for k in range(h.npatches)]
        self.nlevels = 1 + max(h.patches[k].level for k in range(h.npatches))
        handle = ctypes.c_void_p()
        B.check(lib().td_plan_create_quantity(ctx.handle, ctypes.byref(h), _DT[dtype],
                                              _QUANTITY[quantity], ctypes.byref(handle)),
                "td_plan_create_quantity")
        self.handle = handle
        torch = _torch()
        self.torch_dtype = torch.float32 if dtype == "f32" else torch.float64

    @property
    def cells(self) -> int:
        return sum(n * n for n in self.sizes)

    def footprint(self):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        B.check(lib().td_plan_footprint(self.handle, ctypes.byref(a), ctypes.byref(b)),
                "td_plan_footprint")
        return a.value, b.value

    def traffic(self, slopes="given"):
        """{pass: algorithmic HBM bytes per solve} for requests with this
        slopes mode."""
        b = (ctypes.c_double * len(Context.PASSES))()
        B.check(lib().td_plan_traffic(self.handle, _SLOPES[slopes], b), "td_plan_traffic")
        return {p: b[i] for i, p in enumerate(Context.PASSES)}

    def close(self):
        if getattr(self, "handle", None):
            B.check(lib().td_plan_destroy(self.handle), "td_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def outputs(self):
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        fx = [torch.empty((n, n), dtype=self.torch_dtype, device=dev) for n in self.sizes]
        if self.quantity == "potential":
            return fx, None
        fy = [torch.empty((n, n), dtype=self.torch_dtype, device=dev) for n in self.sizes]
        return fx, fy

    def request(self, sigma, dsdx=None, dsdy=None, fx=None, fy=None, slopes="given"):
        """slopes: "given" (dsdx / dsdy as passed, None = zero) or "estimate"
        (TD_SLOPES_ESTIMATE: from sigma on the device; pass no slopes)."""
        mode = _SLOPES.get(slopes)
        if mode is None:
            raise ValueError(f"slopes must be one of {sorted(_SLOPES)}")
        _check_fields(self, sigma, "sigma")
        _check_fields(self, dsdx, "dsdx", required=False)
        _check_fields(self, dsdy, "dsdy", required=False)
        pot = self.quantity == "potential"
        if fx is None or (fy is None and not pot):
            fx, fy = self.outputs()
        _check_fields(self, fx, "fx")
        _check_fields(self, fy, "fy", required=not pot)
        req = B.make_request(self.handle, sigma, dsdx, dsdy, fx, fy, mode)
        req._tensors = (sigma, dsdx, dsdy, fx, fy)
        return req, fx, fy

    def solve(self, sigma, dsdx=None, dsdy=None, fx=None, fy=None, stream=None,
              slopes="given"):
        """Enqueue td_solve on the current (or given) torch stream; returns
        (fx, fy) lists.  Asynchronous: synchronise before reading."""
        req, fx, fy = self.request(sigma, dsdx, dsdy, fx, fy, slopes)
        B.check(lib().td_solve(ctypes.byref(req), _stream_handle(stream)), "td_solve")
        return fx, fy


class Batch:
    """td_batch: many plans solved by one launch per pass and length."""

    def __init__(self, ctx: Context, plans: Sequence[Plan]):
        self.ctx = ctx
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
        h = ctypes.c_void_p()
        B.check(lib().td_batch_create(ctx.handle, len(plans), arr, ctypes.byref(h)),
                "td_batch_create")
        self.handle = h

    def solve(self, fields: List[tuple], outs: Optional[List[tuple]] = None,
              use_graph: bool = False, stream=None):
        """fields[k] = (sigma, dsdx, dsdy[, slopes]) for plan k; returns
        [(fx, fy)]."""
        reqs = (B.td_request * len(self.plans))()
        keep, res = [], []
        for k, (p, f) in enumerate(zip(self.plans, fields)):
            fx, fy = (outs[k] if outs is not None else (None, None))
            r, fx, fy = p.request(f[0], f[1], f[2], fx, fy, f[3] if len(f) > 3 else "given")
            keep.append(r)
            reqs[k] = r
            res.append((fx, fy))
        self._keep = (keep, reqs)
        B.check(lib().td_batch_solve(self.handle, reqs, 1 if use_graph else 0,
                                     _stream_handle(stream)), "td_batch_solve")
        return res

    def set_launch(self, mode: str):
        """Column-pass launches: 'direct' (default: one workgroup per job)
        or 'persistent' (work lists per XCD, about one wave of resident
        workgroups per launch)."""
        m = {"direct": B.TD_LAUNCH_DIRECT, "persistent": B.TD_LAUNCH_PERSISTENT}[mode]
        B.check(lib().td_batch_set_launch(self.handle, m), "td_batch_set_launch")

    def footprint(self) -> int:
        a = ctypes.c_size_t()
        B.check(lib().td_batch_footprint(self.handle, ctypes.byref(a)), "td_batch_footprint")
        return a.value

    def close(self):
        if getattr(self, "handle", None):
            B.check(lib().td_batch_destroy(self.handle), "td_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """td_server: continuous batching of submitted solves."""

    def __init__(self, ctx: Context, max_inflight: int = 2, max_batch: int = 16):
        self.ctx = ctx
        h = ctypes.c_void_p()
        B.check(lib().td_server_create(ctx.handle, max_inflight, max_batch, ctypes.byref(h)),
                "td_server_create")
        self.handle = h
        self._live = {}

    def set_queue_limit(self, max_queued: int):
        B.check(lib().td_server_set_queue_limit(self.handle, max_queued),
                "td_server_set_queue_limit")

    def submit(self, plan: Plan, sigma, dsdx=None, dsdy=None, fx=None, fy=None,
               queue_if_full: bool = True, slopes="given", stream=None):
        """Submit a solve of `plan`.  The solve waits for the work enqueued on
        `stream` (default: the current torch stream) before the call, so
        inputs written there are visible; the tensors are held until the
        ticket is reported done."""
        req, fx, fy = plan.request(sigma, dsdx, dsdy, fx, fy, slopes)
        t = ctypes.c_uint64()
        B.check(lib().td_server_submit(self.handle, ctypes.byref(req), 1 if queue_if_full else 0,
                                       _stream_handle(stream), ctypes.byref(t)),
                "td_server_submit")
        self._live[t.value] = req
        return t.value, fx, fy

    def submit_hierarchy(self, hier, dtype: str, sigma, dsdx=None, dsdy=None, fx=None,
                         fy=None, queue_if_full: bool = True, slopes="given",
                         quantity: str = "force", stream=None):
        """Submit a solve of a hierarchy the caller has no plan for: the
        server plans it (off its launch thread, once per distinct
        hierarchy) and then admits it like any other request."""
        mode = _SLOPES.get(slopes)
        if mode is None:
            raise ValueError(f"slopes must be one of {sorted(_SLOPES)}")
        torch = _torch()
        tdt = torch.float32 if dtype == "f32" else torch.float64
        sizes = [p.n for p in hier.patches]
        pot = quantity == "potential"

        def chk(arrays, name, required):
            if arrays is None:
                if required:
                    raise ValueError(f"{name} is required")
                return
            if len(arrays) != len(sizes):
                raise ValueError(f"{name}: expected {len(sizes)} arrays")
            for t, n in zip(arrays, sizes):
                if t is None:
                    if required:
                        raise ValueError(f"{name} has a None entry")
                    continue
                if not t.is_cuda or t.dtype != tdt or tuple(t.shape) != (n, n) \
                        or not t.is_contiguous():
                    raise ValueError(f"{name}: contiguous {tdt} CUDA tensors of shape (n, n)")
        chk(sigma, "sigma", True)
        chk(dsdx, "dsdx", False)
        chk(dsdy, "dsdy", False)
        if fx is None:
            dev = torch.device("cuda", self.ctx.device)
            fx = [torch.empty((n, n), dtype=tdt, device=dev) for n in sizes]
            fy = None if pot else [torch.empty((n, n), dtype=tdt, device=dev) for n in sizes]
        chk(fx, "fx", True)
        chk(fy, "fy", not pot)
        h = B.make_hierarchy(hier)
        req = B.make_request(None, sigma, dsdx, dsdy, fx, fy, mode)
        req._tensors = (sigma, dsdx, dsdy, fx, fy, h)
        t = ctypes.c_uint64()
        B.check(lib().td_server_submit_hierarchy(self.handle, ctypes.byref(h), _DT[dtype],
                                                 _QUANTITY[quantity], ctypes.byref(req),
                                                 1 if queue_if_full else 0,
                                                 _stream_handle(stream), ctypes.byref(t)),
                "td_server_submit_hierarchy")
        self._live[t.value] = req
        return t.value, fx, fy

    def poll(self, ticket: int):
        """(done, latency_s).  A ticket is reported done once: the server
        then forgets it (polling it again raises TD_EINVAL)."""
        d, lat = ctypes.c_int32(), ctypes.c_double()
        try:
            B.check(lib().td_server_poll(self.handle, ticket, ctypes.byref(d),
                                         ctypes.byref(lat)), "td_server_poll")
        except TdError:
            self._live.pop(ticket, None)
            raise
        if d.value:
            self._live.pop(ticket, None)
        return bool(d.value), lat.value

    def cancel(self, ticket: int):
        B.check(lib().td_server_cancel(self.handle, ticket), "td_server_cancel")
        self._live.pop(ticket, None)

    def drain(self):
        B.check(lib().td_server_drain(self.handle), "td_server_drain")

    def stats(self):
        v = [ctypes.c_uint64() for _ in range(6)]
        B.check(lib().td_server_stats(self.handle, *[ctypes.byref(x) for x in v]),
                "td_server_stats")
        out = dict(zip(["completed", "cancelled", "refused", "deferred", "batches",
                        "peak_queue"], [x.value for x in v]))
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        B.check(lib().td_server_stats2(self.handle, ctypes.byref(a), ctypes.byref(b)),
                "td_server_stats2")
        out["planned"] = a.value
        out["failed"] = b.value
        return out

    def close(self):
        if getattr(self, "handle", None):
            B.check(lib().td_server_destroy(self.handle), "td_server_destroy")
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
