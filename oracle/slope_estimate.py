"""In-cell slopes from cell values -- TEST INFRASTRUCTURE ONLY (part of the
oracle; only tests, the smoke check and the CPU-baseline leg use it).

The reconstruction of Section 2.1 (eq. eqnSigma) takes sigma linear in each
cell, with x- and y-slopes that are constants of the cell, and leaves open
how those constants are obtained.  The estimate written out here is the
plain one that reproduces the error tables of Section 3 (Tables 1-5, every
column, at N = 32 and 64):

  * inside a patch, the centred difference of the neighbouring cell values,
        dsdx[j][i] = (s[j][i+1] - s[j][i-1]) / (2 h);
  * in the first and last column (row) of a patch, the one-sided difference
    towards the interior, (s[j][1] - s[j][0]) / h and
    (s[j][n-1] - s[j][n-2]) / h;
  * a patch one cell wide has slope 0 along that axis.

Every patch is treated on its own: values of other patches, of the parent
level, or outside the patch never enter.  Cells covered by a finer patch
keep their stored value here; it enters the slopes of their active
neighbours (it is excluded from the force sum only as a source).
"""
from __future__ import annotations

import numpy as np


def _diff_along(s: np.ndarray, h: float, axis: int) -> np.ndarray:
    """Centred differences along ``axis``, one-sided at both ends."""
    s = np.moveaxis(np.asarray(s, dtype=np.float64), axis, 0)
    n = s.shape[0]
    d = np.zeros_like(s)
    if n >= 2:
        d[1:-1] = (s[2:] - s[:-2]) / (2.0 * h)
        d[0] = (s[1] - s[0]) / h
        d[-1] = (s[-1] - s[-2]) / h
    return np.moveaxis(d, 0, axis)


def slopes(hier, sigma):
    """(dsdx, dsdy): one float64 [n][n] array per patch, row-major [y][x] like
    ``sigma``; h is the patch's own cell width (x) or height (y)."""
    dsdx, dsdy = [], []
    for p, s in zip(hier.patches, sigma):
        dsdx.append(_diff_along(s, hier.h(p.level), axis=1))
        dsdy.append(_diff_along(s, hier.h(p.level) * getattr(hier, "aspect", 1.0), axis=0))
    return dsdx, dsdy
