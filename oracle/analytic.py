"""Potential-density pairs of the generalized Maclaurin disks -- TEST
INFRASTRUCTURE ONLY (part of the oracle).

Appendix of the paper: surface density sigma0 (1 - R^2/alpha^2)^(n - 1/2)
(disk D_n), G = 1.  The potential follows from the recursion eqnPhiDnp1,

    Phi_{D_{n+1}}(R; alpha) = (2n+1)/alpha^(2n+1) int_0^alpha a^(2n) Phi_{D_n}(R; a) da,

started from the Maclaurin potential Phi_{D_1}, or from the closed form
eqnPhiDn with the coefficients b_{n,k}, c_{n,k}.

Reading: in the printed b_{n+1,0}, the middle sum's denominator 2k+1 is taken
as 2k+2 (the same expression as c_{n+1,0}); with it the closed form agrees
with the recursion to working precision, and the pins in the tests check
exactly that.  Everything is evaluated with mpmath at ``DPS`` digits.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import mpmath as mp

DPS = 40


def H(k: int, m: int) -> Fraction:
    """H(k, m) = (-1)^(k-m) prod_{j=m}^{k} (2j+1)/(2j+2)."""
    out = Fraction(1)
    for j in range(m, k + 1):
        out *= Fraction(2 * j + 1, 2 * j + 2)
    return out if (k - m) % 2 == 0 else -out


@lru_cache(maxsize=None)
def coefficients(n: int):
    """(b_{n,0..n}, c_{n,0..n-1}) as exact fractions (appendix recursion)."""
    if n < 1:
        raise ValueError("n >= 1")
    b = [Fraction(1), Fraction(2)]
    c = [Fraction(1)]
    for nn in range(1, n):
        A = b[nn] / (2 * nn + 2) + c[nn - 1]
        nb = [Fraction(0)] * (nn + 2)
        nc = [Fraction(0)] * (nn + 1)
        for k in range(1, nn + 2):
            nb[k] = b[k - 1] / (2 * k)
        mid = sum(((b[k] / (2 * k + 2) + c[k] + c[k - 1]) * H(k, 0) for k in range(1, nn)),
                  Fraction(0))
        nb[0] = A * H(nn, 0) + mid + (b[0] / 4 + c[0] / 2)
        nc[0] = nb[0]
        nc[nn] = A * H(nn, nn) / (2 * nn + 1)
        for m in range(1, nn):
            s = A * H(nn, m) / (2 * m + 1)
            for k in range(m, nn):
                s += (b[k] / (2 * k + 2) + c[k] + c[k - 1]) * H(k, m) / (2 * m + 1)
            nc[m] = s
        b, c = nb, nc
    return tuple(b), tuple(c)


def _prod_odd(n: int) -> int:
    p = 1
    for j in range(n):
        p *= 2 * j + 1
    return p


def potential(n: int, R, alpha, sigma0=1):
    """Phi_{D_n}(R, z=0; alpha), closed form (eq. eqnPhiDn and the interior
    form that follows it)."""
    with mp.workdps(max(DPS, mp.mp.dps)):
        R = mp.mpf(R)
        alpha = mp.mpf(alpha)
        b, c = coefficients(n)
        pre = mp.mpf(_prod_odd(n)) / alpha ** (2 * n - 1)
        if R <= alpha:
            # R^{2n} (xi^2 - 1)^k = R^{2n-2k} (alpha^2 - R^2)^k, a polynomial.
            s = mp.fsum(mp.mpf(b[k].numerator) / b[k].denominator * R ** (2 * n - 2 * k)
                        * (alpha ** 2 - R ** 2) ** k for k in range(n + 1))
            return -mp.pi ** 2 * sigma0 / 4 * pre * s
        xi = alpha / R
        w = xi ** 2 - 1
        sb = mp.fsum(mp.mpf(b[k].numerator) / b[k].denominator * w ** k for k in range(n + 1))
        sc = mp.fsum(mp.mpf(c[k].numerator) / c[k].denominator * w ** k for k in range(n))
        return (-mp.pi * sigma0 / 2 * pre * R ** (2 * n)
                * (sb * mp.asin(xi) + xi * sc * mp.sqrt(1 - xi ** 2)))


def maclaurin_potential(R, alpha, sigma0=1):
    """Phi_{D_1}, the Maclaurin potential as printed in the appendix."""
    with mp.workdps(max(DPS, mp.mp.dps)):
        R = mp.mpf(R)
        alpha = mp.mpf(alpha)
        if R <= alpha:
            return -mp.pi ** 2 * sigma0 / (4 * alpha) * (2 * alpha ** 2 - R ** 2)
        return -mp.pi * sigma0 / (2 * alpha) * ((2 * alpha ** 2 - R ** 2) * mp.asin(alpha / R)
                                                + alpha * mp.sqrt(R ** 2 - alpha ** 2))


def potential_by_recursion(n: int, R, alpha, sigma0=1):
    """Phi_{D_n} from Phi_{D_1} by repeated numerical quadrature of the
    defining recursion eqnPhiDnp1 (independent of the closed form)."""
    with mp.workdps(DPS):
        R = mp.mpf(R)
        alpha = mp.mpf(alpha)

        def phi(k, a):
            if k == 1:
                return maclaurin_potential(R, a, sigma0)
            pts = [0, a] if R >= a else [0, R, a]
            return (2 * k - 1) / a ** (2 * k - 1) * mp.quad(
                lambda t: t ** (2 * k - 2) * phi(k - 1, t), pts)
        return phi(n, alpha)


def radial_force(n: int, R, alpha, sigma0=1):
    """F_R = -dPhi/dR of the D_n disk (G = 1)."""
    with mp.workdps(DPS):
        return -mp.diff(lambda r: potential(n, r, alpha, sigma0), mp.mpf(R))


def force_xy(n: int, x, y, alpha, sigma0=1, cx=0.0, cy=0.0):
    """(F_x, F_y) of a D_n disk centred at (cx, cy), as float64 arrays."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    fx = np.zeros(x.shape)
    fy = np.zeros(x.shape)
    it = np.nditer([x, y], flags=["multi_index"])
    cache = {}
    for xv, yv in it:
        dx, dy = float(xv) - cx, float(yv) - cy
        R = (dx * dx + dy * dy) ** 0.5
        if R == 0:
            continue
        f = cache.get(R)
        if f is None:
            f = float(radial_force(n, R, alpha, sigma0))
            cache[R] = f
        fx[it.multi_index] = f * dx / R
        fy[it.multi_index] = f * dy / R
    return fx, fy


def disk_mass(n: int, alpha, sigma0=1):
    """Total mass 2 pi sigma0 alpha^2 / (2n + 1)."""
    with mp.workdps(DPS):
        return 2 * mp.pi * sigma0 * mp.mpf(alpha) ** 2 / (2 * n + 1)
