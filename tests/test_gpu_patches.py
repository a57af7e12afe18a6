"""Several patches per level (Section 2.1: the grids Omega^l_k, k > 0), through
the C ABI: parity with the oracle on random multi-patch hierarchies and on
the paper's Examples 3 and 4 (two sigma_{D5} disks, alpha = sqrt(2)/4, at
(+-1/2, 0)).  Their error tables are reproduced with the other convergence
tables of Section 3 in the convergence module."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import covered_are_zero, gpu_solve, rand_fields, rel_l2_full

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = synth.TWO_DISK_ALPHA


@pytest.fixture(scope="module")
def ctx():
    import paper_1603_03142_amd as td
    c = td.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def radial():
    from scipy.interpolate import CubicSpline
    from oracle import analytic
    ri = np.linspace(0.0, ALPHA, 1201)
    ro = np.linspace(ALPHA, 2.0, 3601)
    fi = np.array([float(analytic.radial_force(5, r, ALPHA)) if r > 0 else 0.0 for r in ri])
    fo = np.array([float(analytic.radial_force(5, r, ALPHA)) for r in ro])
    si, so = CubicSpline(ri, fi), CubicSpline(ro, fo)
    return lambda r: np.where(r <= ALPHA, si(np.minimum(r, ALPHA)), so(np.maximum(r, ALPHA)))


SEEDS = [(s, [16, 24, 36, 40][s % 4], 2 + s % 3, 1 + s % 3, [2, 4, 3][s % 3]) for s in range(3, 12)]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_random_patches_parity(ctx, dtype, tol):
    """Random fields on random multi-patch hierarchies (ratios 2, 3, 4), full
    field."""
    multi = 0
    for seed, n0, levels, per, ratio in SEEDS:
        hier = synth.random_patches(seed, n0=n0, levels=levels, per_level=per, ratio=ratio)
        multi += any(sum(p.level == l for p in hier.patches) > 1 for l in range(4))
        sig, dx, dy = rand_fields(hier, 50 + seed)
        ox, oy = oracle.forces(hier, sig, dx, dy)
        gx, gy = gpu_solve(ctx, hier, sig, dx, dy, dtype)
        err = rel_l2_full(hier, gx, gy, ox, oy)
        assert err <= tol, (seed, [(p.level, p.n, p.ox, p.oy) for p in hier.patches], err)
        assert covered_are_zero(hier, gx, gy)
    assert multi >= 4


def test_random_patches_estimated_slopes(ctx):
    """Slopes estimated from sigma on multi-patch hierarchies: every patch
    uses its own values only, one-sided at its own edges (patches of one
    level that touch do not see each other)."""
    for seed, n0, levels, per, ratio in SEEDS[:5]:
        hier = synth.random_patches(seed, n0=n0, levels=levels, per_level=per, ratio=ratio)
        sig, _, _ = rand_fields(hier, 70 + seed, slopes=False)
        dx, dy = oracle.slopes(hier, sig)
        ox, oy = oracle.forces(hier, sig, dx, dy)
        gx, gy = gpu_solve(ctx, hier, sig, None, None, "f64", slopes="estimate")
        assert rel_l2_full(hier, gx, gy, ox, oy) <= 1e-12, seed


@pytest.mark.parametrize("example", [3, 4])
def test_examples_vs_oracle(ctx, example):
    hier = synth.example_hierarchy(example, 32)
    sig, dx, dy = synth.sample_fields(hier, synth.two_disks(), "analytic", synth.two_disks_gradient())
    ox, oy = oracle.forces(hier, sig, dx, dy)
    gx, gy = gpu_solve(ctx, hier, sig, dx, dy, "f64")
    assert rel_l2_full(hier, gx, gy, ox, oy) <= 1e-12
