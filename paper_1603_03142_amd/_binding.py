"""ctypes binding of libthindisk.so (argument marshalling only).

Every function here forwards to the C entry point of the same name in
``include/thindisk.h``; device buffers are PyTorch tensors on the GPU whose
``data_ptr()`` is passed through.  There is no fallback: if the HIP library
is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libthindisk.so")

TD_OK, TD_EINVAL, TD_EALIGN, TD_ENEST, TD_ENOMEM, TD_EDEVICE, TD_EBUSY, TD_EUNSUPPORTED = range(8)
TD_F32, TD_F64 = 0, 1
TD_SLOPES_GIVEN, TD_SLOPES_ESTIMATE = 0, 1
TD_FORCE, TD_POTENTIAL = 0, 1
TD_DEBUG_NONFINITE = 1
TD_LAUNCH_DIRECT, TD_LAUNCH_PERSISTENT = 0, 1
TD_MAX_LEVELS = 8
TD_MAX_PATCHES = 8

# Every entry point the header declares.
EXPORTS = [
    "td_context_create", "td_context_destroy", "td_context_usage", "td_context_set_debug",
    "td_debug_nonfinite", "td_hierarchy_check",
    "td_hierarchy_snap", "td_plan_check", "td_plan_create", "td_plan_create_quantity",
    "td_plan_footprint", "td_plan_destroy", "td_solve", "td_solve_noalloc",
    "td_batch_create", "td_batch_solve", "td_batch_footprint", "td_batch_set_launch",
    "td_batch_destroy",
    "td_autotune", "td_timing_enable", "td_timing_read", "td_plan_traffic", "td_server_create", "td_server_set_queue_limit", "td_server_submit",
    "td_server_submit_hierarchy", "td_server_stats2", "td_server_poll", "td_server_drain",
    "td_server_cancel", "td_server_stats", "td_server_destroy", "td_kernel_table",
    "td_status_string", "td_last_error", "td_version",
]


class TdError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


_STATUS = {0: "TD_OK", 1: "TD_EINVAL", 2: "TD_EALIGN", 3: "TD_ENEST", 4: "TD_ENOMEM",
           5: "TD_EDEVICE", 6: "TD_EBUSY", 7: "TD_EUNSUPPORTED"}


class td_patch(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("n", ctypes.c_int32), ("ox", ctypes.c_int32),
                ("oy", ctypes.c_int32)]


class td_hierarchy(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("h0", ctypes.c_double),
                ("ratio", ctypes.c_int32), ("npatches", ctypes.c_int32),
                ("patches", ctypes.POINTER(td_patch)), ("aspect", ctypes.c_double)]


VP = ctypes.c_void_p
VPP = ctypes.POINTER(ctypes.c_void_p)


class td_request(ctypes.Structure):
    _fields_ = [("plan", VP), ("sigma", VPP), ("dsdx", VPP), ("dsdy", VPP), ("fx", VPP),
                ("fy", VPP), ("slopes", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is not built; run "
                              "`python -m paper_1603_03142_amd.build` (no CPU fallback exists)")
        # Load PyTorch's HIP runtime first: the library's libamdhip64.so.7
        # dependency then binds to that same runtime, so device memory and
        # streams from torch are valid in both (one runtime per process).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        S = ctypes.c_int
        sz = ctypes.POINTER(ctypes.c_size_t)
        u64 = ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "td_context_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(VP)], S),
            "td_context_destroy": ([VP], S),
            "td_context_usage": ([VP, sz, sz], S),
            "td_context_set_debug": ([VP, ctypes.c_int32], S),
            "td_debug_nonfinite": ([VP, u64], S),
            "td_hierarchy_check": ([ctypes.POINTER(td_hierarchy)], S),
            "td_hierarchy_snap": ([ctypes.POINTER(td_hierarchy), ctypes.POINTER(td_patch),
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)], S),
            "td_plan_create": ([VP, ctypes.POINTER(td_hierarchy), ctypes.c_int,
                                ctypes.POINTER(VP)], S),
            "td_plan_create_quantity": ([VP, ctypes.POINTER(td_hierarchy), ctypes.c_int,
                                         ctypes.c_int32, ctypes.POINTER(VP)], S),
            "td_plan_footprint": ([VP, sz, sz], S),
            "td_plan_check": ([ctypes.POINTER(td_hierarchy), ctypes.c_int, sz], S),
            "td_plan_destroy": ([VP], S),
            "td_solve": ([ctypes.POINTER(td_request), VP], S),
            "td_solve_noalloc": ([ctypes.POINTER(td_request), VP], S),
            "td_batch_create": ([VP, ctypes.c_int32, ctypes.POINTER(VP), ctypes.POINTER(VP)], S),
            "td_batch_solve": ([VP, ctypes.POINTER(td_request), ctypes.c_int, VP], S),
            "td_batch_footprint": ([VP, sz], S),
            "td_batch_set_launch": ([VP, ctypes.c_int32], S),
            "td_batch_destroy": ([VP], S),
            "td_autotune": ([VP, ctypes.c_int, ctypes.c_int32, ctypes.c_char_p], S),
            "td_server_create": ([VP, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(VP)], S),
            "td_server_set_queue_limit": ([VP, ctypes.c_int32], S),
            "td_server_submit": ([VP, ctypes.POINTER(td_request), ctypes.c_int32, VP, u64], S),
            "td_server_submit_hierarchy": ([VP, ctypes.POINTER(td_hierarchy), ctypes.c_int,
                                            ctypes.c_int32, ctypes.POINTER(td_request),
                                            ctypes.c_int32, VP, u64], S),
            "td_server_stats2": ([VP, u64, u64], S),
            "td_server_poll": ([VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_double)], S),
            "td_server_drain": ([VP], S),
            "td_server_cancel": ([VP, ctypes.c_uint64], S),
            "td_server_stats": ([VP, u64, u64, u64, u64, u64, u64], S),
            "td_server_destroy": ([VP], S),
            "td_kernel_table": ([VP, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_double)], S),
            "td_timing_enable": ([VP, ctypes.c_int], S),
            "td_timing_read": ([VP, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64)], S),
            "td_plan_traffic": ([VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)], S),
            "td_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "td_last_error": ([], ctypes.c_char_p),
            "td_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != TD_OK:
        raise TdError(status, where, lib().td_last_error().decode())


def make_hierarchy(hier):
    """td_hierarchy from an object with x0, y0, h0, ratio and either
    ``patches`` (level/n/ox/oy, grouped by level, level 0 first -- the order
    of every per-patch array) or ``levels`` ((n, ox, oy), one patch per
    level)."""
    if hasattr(hier, "patches"):
        pats = [(p.level, p.n, p.ox, p.oy) for p in hier.patches]
        if [p[0] for p in pats] != sorted(p[0] for p in pats):
            raise ValueError("patches must be grouped by level, level 0 first")
    else:
        pats = [(l, n, ox, oy) for l, (n, ox, oy) in enumerate(hier.levels)]
    arr = (td_patch * len(pats))(*[td_patch(*p) for p in pats])
    h = td_hierarchy(float(hier.x0), float(hier.y0), float(hier.h0), int(hier.ratio), len(pats),
                     ctypes.cast(arr, ctypes.POINTER(td_patch)),
                     float(getattr(hier, "aspect", 1.0)))
    h._keep = arr
    return h


def _ptr_array(tensors: Optional[Sequence]):
    if tensors is None:
        return None, None
    arr = (VP * len(tensors))(*[VP(t.data_ptr()) if t is not None else VP(0) for t in tensors])
    return ctypes.cast(arr, VPP), arr


def make_request(plan_handle, sigma, dsdx, dsdy, fx, fy, slopes=TD_SLOPES_GIVEN):
    keep = []
    ps, a = _ptr_array(sigma); keep.append(a)
    px, a = _ptr_array(dsdx); keep.append(a)
    py, a = _ptr_array(dsdy); keep.append(a)
    pfx, a = _ptr_array(fx); keep.append(a)
    pfy, a = _ptr_array(fy); keep.append(a)
    r = td_request(plan_handle, ps, px, py, pfx, pfy, slopes)
    r._keep = keep
    return r
