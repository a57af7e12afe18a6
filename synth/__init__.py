"""Seeded synthetic inputs for the thin-disk force solver.

This module holds input generation only: grid hierarchies, surface-density
functions, their sampling onto cell centres and the slope estimates handed to
the solver.  It contains none of the force method's arithmetic, and both the
oracle and the HIP path consume what it produces.

Geometry convention (Section 2.1 of the paper): patch p lives on level
``level``; its cells have side ``h0 / ratio**level``; its lower-left corner is
``(x0 + ox*h, y0 + oy*h)`` where ``ox, oy`` are integer offsets in the patch's
own cell units from the level-0 origin.  Fields are row-major ``[j][i]`` with
x fastest.

Workload recipes (stand-ins for the paper's sigma_{D_n} experiments, Section 3
and the appendix; the paper uses no public dataset):
  * disk family sigma_{D_n}(r; alpha) = sigma0 (1 - r^2/alpha^2)^(n - 1/2);
  * Gaussian clump amp * exp(-d^2 / (2 w^2));
  * lognormal perturbation exp(g), g a random-Fourier-mode sample of a
    zero-mean field with squared-exponential covariance;
  * slopes by the central difference of the analytic sigma at x +- h.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Patch", "Hierarchy", "disk_dn", "clump", "LognormalField", "sample_fields",
    "cell_centres", "covered_mask", "sample_targets", "config1", "config2", "config3",
    "config4", "config5_requests", "nested_hierarchy", "snap_offsets", "example_hierarchy",
    "two_disks", "two_disks_gradient", "random_patches",
]


@dataclasses.dataclass(frozen=True)
class Patch:
    level: int
    n: int
    ox: int
    oy: int


@dataclasses.dataclass
class Hierarchy:
    x0: float
    y0: float
    h0: float
    ratio: int
    patches: List[Patch]
    aspect: float = 1.0  # cell height / cell width, the same on every level

    @property
    def nlevels(self) -> int:
        return 1 + max(p.level for p in self.patches)

    def h(self, level: int) -> float:
        """Cell width (x side) on ``level``."""
        return self.h0 / (self.ratio ** level)

    def hy(self, level: int) -> float:
        """Cell height (y side) on ``level``."""
        return self.h(level) * self.aspect

    def lower_left(self, p: Patch) -> Tuple[float, float]:
        return self.x0 + p.ox * self.h(p.level), self.y0 + p.oy * self.hy(p.level)

    @property
    def cells(self) -> int:
        return sum(p.n * p.n for p in self.patches)

    def one_patch_per_level(self) -> bool:
        levels = [p.level for p in self.patches]
        return levels == list(range(len(levels)))


def nested_hierarchy(x0: float, y0: float, h0: float, ratio: int,
                     levels: Sequence[Tuple[int, int, int]], aspect: float = 1.0) -> Hierarchy:
    """One patch per level; ``levels[l] = (n, ox, oy)``."""
    return Hierarchy(x0, y0, h0, ratio,
                     [Patch(l, n, ox, oy) for l, (n, ox, oy) in enumerate(levels)], aspect)


def snap_offsets(x0: float, y0: float, h0: float, ratio: int, n_levels: Sequence[int],
                 centres: Sequence[Tuple[float, float]]) -> List[Tuple[int, int, int]]:
    """Place level l >= 1 (n_levels[l] cells, one patch per level) as close as
    the parent lattice allows to a requested centre: the lower-left corner is
    rounded to the nearest parent node and clamped inside the parent.
    ``centres[l-1]`` is the requested centre of level l."""
    out = [(n_levels[0], 0, 0)]
    h = h0
    for l in range(1, len(n_levels)):
        n = n_levels[l]
        pn, pox, poy = out[-1]
        if n % ratio:
            raise ValueError("child patch width must be a multiple of the ratio")
        span = n // ratio  # parent cells covered by the child
        if span > pn:
            raise ValueError("child patch wider than its parent")
        px0, py0 = x0 + pox * h, y0 + poy * h
        cx, cy = centres[l - 1]
        ext = n * h / ratio
        kx = math.floor((cx - ext / 2 - px0) / h + 0.5)
        ky = math.floor((cy - ext / 2 - py0) / h + 0.5)
        kx = min(max(kx, 0), pn - span)
        ky = min(max(ky, 0), pn - span)
        out.append((n, ratio * (pox + kx), ratio * (poy + ky)))
        h /= ratio
    return out


# ----------------------------------------------------------------------------
# surface densities
# ----------------------------------------------------------------------------

def disk_dn(n: int, alpha: float, sigma0: float = 1.0, cx: float = 0.0, cy: float = 0.0):
    """sigma_{D_n}(r; alpha) of Section 3 (generalized Maclaurin disk)."""
    def f(x, y):
        r2 = (np.asarray(x) - cx) ** 2 + (np.asarray(y) - cy) ** 2
        q = np.clip(1.0 - r2 / (alpha * alpha), 0.0, None)
        return np.where(r2 < alpha * alpha, sigma0 * q ** (n - 0.5), 0.0)
    return f


def disk_dn_gradient(n: int, alpha: float, sigma0: float = 1.0, cx: float = 0.0,
                     cy: float = 0.0):
    """Analytic gradient of sigma_{D_n} (finite for n >= 2 at the edge)."""
    def g(x, y):
        dx = np.asarray(x) - cx
        dy = np.asarray(y) - cy
        r2 = dx * dx + dy * dy
        inside = r2 < alpha * alpha
        q = np.clip(1.0 - r2 / (alpha * alpha), 0.0, None)
        with np.errstate(divide="ignore", invalid="ignore"):
            fac = np.where(inside, sigma0 * (n - 0.5) * q ** (n - 1.5) * (-2.0 / alpha ** 2), 0.0)
        return fac * dx, fac * dy
    return g


def clump(amp: float, width: float, cx: float, cy: float):
    def f(x, y):
        d2 = (np.asarray(x) - cx) ** 2 + (np.asarray(y) - cy) ** 2
        return amp * np.exp(-d2 / (2.0 * width * width))
    return f


class LognormalField:
    """exp(g): g = std * sqrt(2/K) * sum_k cos(w_k . x + b_k), w_k ~ N(0, I/l^2),
    b_k ~ U[0, 2pi): a K-mode sample of a field with covariance
    std^2 exp(-|d|^2 / (2 l^2)).  Being a continuous function, every level of
    a hierarchy samples the same realisation."""

    def __init__(self, seed: int, std: float, corr_len: float, modes: int = 512):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.w = rng.normal(0.0, 1.0 / corr_len, size=(modes, 2))
        self.b = rng.uniform(0.0, 2.0 * np.pi, size=modes)
        self.amp = std * math.sqrt(2.0 / modes)

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if x.ndim == 2 and x.shape == y.shape and np.all(x == x[:1]) and np.all(y == y[:, :1]):
            # tensor-product grid (rows of x equal, columns of y equal):
            # cos(a + b + c) = Re(e^{ia} e^{ib} e^{ic}) turns the mode sum
            # into one complex matrix product
            ex = np.exp(1j * (np.outer(x[0], self.w[:, 0]) + self.b))
            ey = np.exp(1j * np.outer(y[:, 0], self.w[:, 1]))
            return np.exp(self.amp * (ey @ ex.T).real)
        g = np.zeros(np.broadcast(x, y).shape)
        for k in range(0, len(self.b), 64):
            w = self.w[k:k + 64]
            ph = (x[..., None] * w[:, 0] + y[..., None] * w[:, 1] + self.b[k:k + 64])
            g += np.cos(ph).sum(axis=-1)
        return np.exp(self.amp * g)


def product(*fs):
    def f(x, y):
        out = fs[0](x, y)
        for g in fs[1:]:
            out = out * g(x, y)
        return out
    return f


def total(*fs):
    def f(x, y):
        out = fs[0](x, y)
        for g in fs[1:]:
            out = out + g(x, y)
        return out
    return f


# ----------------------------------------------------------------------------
# sampling onto a hierarchy
# ----------------------------------------------------------------------------

def cell_centres(hier: Hierarchy, p: Patch) -> Tuple[np.ndarray, np.ndarray]:
    xl, yl = hier.lower_left(p)
    i = np.arange(p.n, dtype=np.float64)
    xc = xl + (i + 0.5) * hier.h(p.level)
    yc = yl + (i + 0.5) * hier.hy(p.level)
    X, Y = np.meshgrid(xc, yc)  # [j][i]
    return X, Y


def covered_mask(hier: Hierarchy, p: Patch) -> np.ndarray:
    """True where a patch one level finer covers the cell (geometry only)."""
    m = np.zeros((p.n, p.n), dtype=bool)
    r = hier.ratio
    for c in hier.patches:
        if c.level != p.level + 1:
            continue
        i0 = c.ox // r - p.ox
        j0 = c.oy // r - p.oy
        w = c.n // r
        ia, ib = max(i0, 0), min(i0 + w, p.n)
        ja, jb = max(j0, 0), min(j0 + w, p.n)
        if ia < ib and ja < jb:
            m[ja:jb, ia:ib] = True
    return m


def sample_fields(hier: Hierarchy, sigma_fn: Callable, slopes: str = "central",
                  grad_fn: Optional[Callable] = None):
    """sigma at cell centres and slopes per patch (lists of float64 arrays).

    slopes: "central" -- (sigma(x+h) - sigma(x-h)) / 2h of the analytic
    function with h the cell's own size; "analytic" -- ``grad_fn`` at the
    centre; "none" -- slopes omitted (None)."""
    sig, dx, dy = [], [], []
    for p in hier.patches:
        X, Y = cell_centres(hier, p)
        h, hy = hier.h(p.level), hier.hy(p.level)
        sig.append(np.ascontiguousarray(sigma_fn(X, Y), dtype=np.float64))
        if slopes == "central":
            dx.append(np.ascontiguousarray((sigma_fn(X + h, Y) - sigma_fn(X - h, Y)) / (2 * h)))
            dy.append(np.ascontiguousarray((sigma_fn(X, Y + hy) - sigma_fn(X, Y - hy)) / (2 * hy)))
        elif slopes == "analytic":
            gx, gy = grad_fn(X, Y)
            dx.append(np.ascontiguousarray(gx, dtype=np.float64))
            dy.append(np.ascontiguousarray(gy, dtype=np.float64))
        elif slopes == "none":
            dx.append(None)
            dy.append(None)
        else:
            raise ValueError(slopes)
    return sig, dx, dy


def sample_targets(hier: Hierarchy, count: int, seed: int, interface_frac: float = 0.25,
                   band: int = 2):
    """Active target cells, stratified by patch, a fraction drawn from the
    band of ``band`` cells next to a level interface (patch edge or covered
    region).  Returns (patch_idx, i, j) int32 arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per = max(1, count // len(hier.patches))
    tp, ti, tj = [], [], []
    for k, p in enumerate(hier.patches):
        act = ~covered_mask(hier, p)
        near = np.zeros_like(act)
        cov = ~act
        # distance-to-interface band: patch edges (for refined levels) and
        # the rim of the covered region.
        if p.level > 0:
            near[:band, :] = near[-band:, :] = True
            near[:, :band] = near[:, -band:] = True
        if cov.any():
            grow = cov.copy()
            for _ in range(band):
                g = grow.copy()
                g[1:, :] |= grow[:-1, :]
                g[:-1, :] |= grow[1:, :]
                g[:, 1:] |= grow[:, :-1]
                g[:, :-1] |= grow[:, 1:]
                grow = g
            near |= grow
        near &= act
        jj_a, ii_a = np.nonzero(act)
        jj_n, ii_n = np.nonzero(near)
        n_near = min(int(round(per * interface_frac)), len(ii_n))
        n_rest = min(per - n_near, len(ii_a))
        if n_near:
            s = rng.choice(len(ii_n), size=n_near, replace=False)
            tp += [k] * n_near
            ti += list(ii_n[s])
            tj += list(jj_n[s])
        if n_rest:
            s = rng.choice(len(ii_a), size=n_rest, replace=False)
            tp += [k] * n_rest
            ti += list(ii_a[s])
            tj += list(jj_a[s])
    return (np.asarray(tp, np.int32), np.asarray(ti, np.int32), np.asarray(tj, np.int32))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def config1():
    """One 64x64 level on [-1,1]^2; Maclaurin disk R = 0.8, sigma0 = 1."""
    hier = nested_hierarchy(-1.0, -1.0, 2.0 / 64, 2, [(64, 0, 0)])
    return hier, disk_dn(1, 0.8)


def config2():
    """Two nested 256x256 levels; level 1 covers [-1/2,1/2]^2 of the [-1,1]^2
    base; Maclaurin R = 0.8 plus a Gaussian clump (amp 5, width 0.03) at
    (0.2, 0.1)."""
    hier = nested_hierarchy(-1.0, -1.0, 2.0 / 256, 2, [(256, 0, 0), (256, 128, 128)])
    return hier, total(disk_dn(1, 0.8), clump(5.0, 0.03, 0.2, 0.1))


def config3():
    """Four nested 512x512 levels (ratio 2, level-l extent 2^(1-l)) centred as
    near (0.3, 0) as the lattices allow; sigma = sigma_{D_2}(R=0.9) times a
    lognormal perturbation (std 0.2, correlation length 4 base cells, seed 3)."""
    h0 = 2.0 / 512
    lv = snap_offsets(-1.0, -1.0, h0, 2, [512] * 4, [(0.3, 0.0)] * 3)
    hier = nested_hierarchy(-1.0, -1.0, h0, 2, lv)
    return hier, product(disk_dn(2, 0.9), LognormalField(3, 0.2, 4 * h0, 512))


def _random_nested(rng, n: int, nlev: int):
    lv = [(n, 0, 0)]
    for _ in range(1, nlev):
        pn, pox, poy = lv[-1]
        span = n // 2
        kx = int(rng.integers(0, pn - span + 1))
        ky = int(rng.integers(0, pn - span + 1))
        lv.append((n, 2 * (pox + kx), 2 * (poy + ky)))
    return nested_hierarchy(-1.0, -1.0, 2.0 / n, 2, lv)


def config4(seed: int = 4, count: int = 64, sizes=(64, 128, 256, 512), max_levels: int = 3):
    """``count`` independent disks: base N from ``sizes``, 1..max_levels nested
    levels of N^2 cells at random aligned positions; sigma_{D_n}, n in 1..5,
    alpha in [0.5, 0.9], centred at the origin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        nlev = int(rng.integers(1, max_levels + 1))
        hier = _random_nested(rng, n, nlev)
        order = int(rng.integers(1, 6))
        alpha = float(rng.uniform(0.5, 0.9))
        out.append((hier, disk_dn(order, alpha)))
    return out


def config5_requests(seed: int = 5, rate: float = 2000.0, duration: float = 10.0,
                     sizes=(128, 256, 512, 1024), max_levels: int = 5):
    """Poisson arrivals (exponential gaps of mean 1/rate): list of
    (arrival_time, hierarchy, sigma_fn).  sigma = sigma_{D_n} (n in 2..5,
    alpha in [0.5, 0.9]) times a lognormal perturbation (std 0.2,
    correlation length 4 base cells)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            break
        n = int(rng.choice(sizes))
        nlev = int(rng.integers(1, max_levels + 1))
        hier = _random_nested(rng, n, nlev)
        order = int(rng.integers(2, 6))
        alpha = float(rng.uniform(0.5, 0.9))
        fseed = int(rng.integers(0, 2 ** 31 - 1))
        out.append((t, hier, (order, alpha, fseed)))
    return out


def request_sigma(order: int, alpha: float, fseed: int, h0: float, modes: int = 128):
    return product(disk_dn(order, alpha), LognormalField(fseed, 0.2, 4 * h0, modes))


def _snap(v: float, h: float) -> int:
    return int(math.floor(v / h + 0.5))


def example_hierarchy(example: int, n: int) -> Hierarchy:
    """Grids of the paper's Examples 1-4 (Section 3), ratio 2, level 0 on
    [-1,1]^2 with N cells per side (h_l = 2^(1-l) / N).
      1: level 1 = [-1/2,1/2]^2 (N cells).
      2: level 1 as in 1, level 2 = [-1/4,1/4]^2 (N cells).
      3: level 1 = [-0.75,-0.25] x [-0.25,0.25] and [0.25,0.75] x [-0.25,0.25]
         (N/2 cells each; N a multiple of 8).
      4: level 2 = the two squares of 3 (N cells each); level 1 = squares of
         side 0.8 around them, [-0.9,-0.1] x [-0.4,0.4] and mirror, whose
         edges lie on no 2^k lattice: each is snapped to the nearest level-0
         nodes (side rounded to a whole number of level-0 cells)."""
    h0 = 2.0 / n
    if example == 1:
        return nested_hierarchy(-1.0, -1.0, h0, 2, [(n, 0, 0), (n, n // 2, n // 2)])
    if example == 2:
        return nested_hierarchy(-1.0, -1.0, h0, 2,
                                [(n, 0, 0), (n, n // 2, n // 2), (n, 3 * n // 2, 3 * n // 2)])
    if example in (3, 4):
        if n % 8:
            raise ValueError("N must be a multiple of 8")
        pats = [Patch(0, n, 0, 0)]
        h1, h2 = h0 / 2, h0 / 4
        if example == 3:
            for x0 in (-0.75, 0.25):
                pats.append(Patch(1, n // 2, _snap(x0 + 1.0, h1), _snap(-0.25 + 1.0, h1)))
            return Hierarchy(-1.0, -1.0, h0, 2, pats)
        side = _snap(0.8, h0)  # level-0 cells
        for x0 in (-0.9, 0.1):
            pats.append(Patch(1, 2 * side, 2 * _snap(x0 + 1.0, h0), 2 * _snap(-0.4 + 1.0, h0)))
        for x0 in (-0.75, 0.25):
            pats.append(Patch(2, n, _snap(x0 + 1.0, h2), _snap(-0.25 + 1.0, h2)))
        return Hierarchy(-1.0, -1.0, h0, 2, pats)
    raise ValueError(example)


TWO_DISKS = ((-0.5, 0.0), (0.5, 0.0))
TWO_DISK_ALPHA = math.sqrt(2.0) / 4


def two_disks(n: int = 5, alpha: float = TWO_DISK_ALPHA):
    """Examples 3-4: two sigma_{D_n} disks centred at (-1/2, 0), (1/2, 0)."""
    return total(*[disk_dn(n, alpha, cx=cx, cy=cy) for cx, cy in TWO_DISKS])


def two_disks_gradient(n: int = 5, alpha: float = TWO_DISK_ALPHA):
    gs = [disk_dn_gradient(n, alpha, cx=cx, cy=cy) for cx, cy in TWO_DISKS]

    def g(x, y):
        ax, ay = gs[0](x, y)
        bx, by = gs[1](x, y)
        return ax + bx, ay + by
    return g


def random_patches(seed: int, n0: int = 32, levels: int = 3, per_level: int = 2,
                   ratio: int = 2, max_patches: int = 8) -> Hierarchy:
    """Several non-overlapping aligned square patches per level, each inside
    one patch of the level above (seeded; at most max_patches in all)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    while ratio ** (levels - 1) > 16:
        levels -= 1
    pats = [Patch(0, n0, 0, 0)]
    parents = [pats[0]]
    for lev in range(1, levels):
        placed = []
        for _ in range(per_level * 8):
            if len(placed) == per_level or len(pats) + len(placed) == max_patches:
                break
            par = parents[int(rng.integers(0, len(parents)))]
            w = int(rng.integers(2, max(3, par.n // 2) + 1))      # parent cells
            kx = int(rng.integers(0, par.n - w + 1))
            ky = int(rng.integers(0, par.n - w + 1))
            cand = Patch(lev, ratio * w, ratio * (par.ox + kx), ratio * (par.oy + ky))
            if all(cand.ox + cand.n <= q.ox or q.ox + q.n <= cand.ox or
                   cand.oy + cand.n <= q.oy or q.oy + q.n <= cand.oy for q in placed):
                placed.append(cand)
        if not placed:
            break
        pats.extend(placed)
        parents = placed
    return Hierarchy(-1.0, -1.0, 2.0 / n0, ratio, pats)
