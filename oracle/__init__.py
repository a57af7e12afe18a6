"""Oracle for the thin-disk force solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does, and this
package never imports the product package: the two share only the seeded
input generators in ``synth``.

Contents:
  * ``direct_sum.c`` -- plain long-double O(cells^2) direct sums of the
    second-order cell-integral formulae (Section 2.1) for the force and for
    the potential, plus the 1-D generalized convolutions of Section 2.2
    written out as sums;
  * ``analytic`` -- potential-density pairs of the generalized Maclaurin
    disks (appendix) for the convergence pins;
  * ``slope_estimate.slopes`` (also ``oracle.slopes``) -- in-cell slopes
    estimated from the cell values (centred differences, one-sided at patch
    edges).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct_sum.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            L.oracle_cell_integrals.argtypes = [ctypes.c_double] * 4 + [dp]
            L.oracle_cell_integrals.restype = None
            L.oracle_forces.argtypes = [ctypes.c_int, ip, ip, ip, ip, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int,
                                        ctypes.POINTER(dp), ctypes.POINTER(dp),
                                        ctypes.POINTER(dp), ctypes.c_int, ip, ip, ip, dp, dp,
                                        ctypes.c_int]
            L.oracle_forces.restype = ctypes.c_int
            L.oracle_cell_potential.argtypes = [ctypes.c_double] * 4 + [dp]
            L.oracle_cell_potential.restype = None
            L.oracle_potential.argtypes = L.oracle_forces.argtypes[:-3] + [dp, ctypes.c_int]
            L.oracle_potential.restype = ctypes.c_int
            L.oracle_genconv1d.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp,
                                           ctypes.c_int, dp, ctypes.c_int]
            L.oracle_genconv1d.restype = None
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def cell_integrals(ua: float, ub: float, va: float, vb: float) -> np.ndarray:
    """[I0, Ixx, Ixy, J0, Jyy, Jyx] of the cell [ua,ub]x[va,vb] relative to a
    target at the origin (Section 2.1, corrected slope antiderivatives)."""
    out = np.zeros(6)
    lib().oracle_cell_integrals(float(ua), float(ub), float(va), float(vb), _dp(out))
    return out


def cell_potential_integrals(ua: float, ub: float, va: float, vb: float) -> np.ndarray:
    """[P0, Px, Py] = integrals of 1/r, (u - uc)/r, (v - vc)/r over the cell
    [ua,ub]x[va,vb] relative to a target at the origin (the potential's
    kernel, eq. eqnPhixy0, with the linear density of eq. eqnSigma)."""
    out = np.zeros(3)
    lib().oracle_cell_potential(float(ua), float(ub), float(va), float(vb), _dp(out))
    return out


def potential(hier, sigma, dsdx=None, dsdy=None, targets=None, nthreads: int = 0):
    """Direct-sum potential Phi = -sum over active source cells of the
    integral of sigma / rho (G = 1).  Arguments as for ``forces``; returns a
    list of phi arrays per patch, or a flat array for ``targets``.  Covered
    targets get 0."""
    return _direct(hier, sigma, dsdx, dsdy, targets, nthreads, potential=True)


def forces(hier, sigma, dsdx=None, dsdy=None, targets=None, nthreads: int = 0):
    """Direct-sum forces.

    ``sigma``/``dsdx``/``dsdy``: one float64 [n][n] array per patch of
    ``hier`` (slopes may be None, or lists holding None).  ``targets``: None
    for every cell of every patch (returns lists of (fx, fy) arrays per
    patch), or a (patch, i, j) triple of int arrays (returns flat fx, fy).
    Covered targets get 0."""
    return _direct(hier, sigma, dsdx, dsdy, targets, nthreads, potential=False)


def _direct(hier, sigma, dsdx, dsdy, targets, nthreads, potential):
    P = len(hier.patches)
    level = np.array([p.level for p in hier.patches], np.int32)
    n = np.array([p.n for p in hier.patches], np.int32)
    ox = np.array([p.ox for p in hier.patches], np.int32)
    oy = np.array([p.oy for p in hier.patches], np.int32)
    keep = []

    def ptrs(arrs):
        if arrs is None or all(a is None for a in arrs):
            return None
        out = (ctypes.POINTER(ctypes.c_double) * P)()
        for k in range(P):
            a = arrs[k]
            if a is None:
                a = np.zeros((hier.patches[k].n,) * 2)
            a = np.ascontiguousarray(a, dtype=np.float64)
            assert a.shape == (hier.patches[k].n,) * 2
            keep.append(a)
            out[k] = _dp(a)
        return out

    ps, px, py = ptrs(sigma), ptrs(dsdx), ptrs(dsdy)
    full = targets is None
    if full:
        tp = np.concatenate([np.full(p.n * p.n, k, np.int32) for k, p in enumerate(hier.patches)])
        ti = np.concatenate([np.tile(np.arange(p.n, dtype=np.int32), p.n) for p in hier.patches])
        tj = np.concatenate([np.repeat(np.arange(p.n, dtype=np.int32), p.n)
                             for p in hier.patches])
    else:
        tp, ti, tj = (np.ascontiguousarray(t, dtype=np.int32) for t in targets)
    fx = np.zeros(len(tp))
    fy = np.zeros(len(tp))
    geo = (P, _ip(level), _ip(n), _ip(ox), _ip(oy), hier.x0, hier.y0, hier.h0,
           float(getattr(hier, "aspect", 1.0)), hier.ratio,
           ps, px, py, len(tp), _ip(tp), _ip(ti), _ip(tj))
    if potential:
        rc = lib().oracle_potential(*geo, _dp(fx), int(nthreads))
    else:
        rc = lib().oracle_forces(*geo, _dp(fx), _dp(fy), int(nthreads))
    if rc != 0:
        raise ValueError("oracle: malformed target list")

    def per_patch(a):
        out, o = [], 0
        for p in hier.patches:
            out.append(a[o:o + p.n * p.n].reshape(p.n, p.n))
            o += p.n * p.n
        return out
    if potential:
        return fx if not full else per_patch(fx)
    return (fx, fy) if not full else (per_patch(fx), per_patch(fy))


def genconv1d(mode: int, m: int, b, c, na: int) -> np.ndarray:
    """Plain sums of the generalized convolutions of Section 2.2 (1-D):
    mode 1 a_n = sum b_{n-k} c_k; mode 2 a_n = sum b_{mn-k} c_k (eq. eqnbmnn);
    mode 3 a_n = sum b_{n-mk} c_k (eq. eqnbnmn)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    a = np.zeros(na)
    lib().oracle_genconv1d(mode, m, _dp(b), len(b), _dp(c), len(c), _dp(a), na)
    return a


from .slope_estimate import slopes  # noqa: E402
