"""GPU path vs the oracle, element by element, through the C ABI.

Tolerances (rel-L2 over active cells, Fx and Fy together): FP64 path 1e-12,
FP32 path 1e-5.  Covered cells must be exactly 0.  Inputs are seeded
synthetic fields from ``synth``; expected values come only from ``oracle``.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import (covered_are_zero, gpu_solve, name_seed, rand_fields, rel_l2,
                         rel_l2_full, sampled)

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import paper_1603_03142_amd as td
    c = td.Context(0)
    yield c
    c.close()


# ---------------------------------------------------------------------------
# kernel tables (FP64 on the GPU) vs the oracle's cell integrals
# ---------------------------------------------------------------------------

TABLE_CASES = [(16, 1, 1, 0, 0), (32, 1, 1, 0, 0), (16, 2, 2, 0, 0), (16, 2, 2, 1, 1),
               (32, 2, 4, 1, 3), (16, 3, 2, 0, 1), (32, 3, 4, 3, 2), (16, 3, 2, 1, 1),
               # odd ratio: half-integer Case-2 offsets, self-mirror middle phase
               (16, 2, 3, 1, 1), (32, 2, 9, 7, 2), (16, 3, 3, 2, 0), (32, 3, 9, 4, 8)]


@pytest.mark.parametrize("M,kind,m,kx,ky", TABLE_CASES)
def test_kernel_table_vs_oracle(ctx, M, kind, m, kx, ky):
    got = ctx.kernel_table(M, kind, m, kx, ky)
    want = np.zeros_like(got)
    for ny in range(M):
        for nx in range(M):
            if nx == M // 2 or ny == M // 2:
                continue
            sx = nx if nx < M // 2 else nx - M
            sy = ny if ny < M // 2 else ny - M
            if kind == 1:
                ua, va, w = -sx - 0.5, -sy - 0.5, 1.0
            elif kind == 2:
                ua, va, w = -m * sx + kx - m / 2, -m * sy + ky - m / 2, 1.0
            else:
                ua, va, w = -m * sx - kx - 0.5, -m * sy - ky - 0.5, float(m)
            c = oracle.cell_integrals(ua, ua + w, va, va + w)
            if kind == 3:
                c[[1, 2, 4, 5]] /= m
            want[:, ny, nx] = c
    assert np.all(np.isfinite(got))
    scale = np.abs(want).max()
    # a few ulp of the largest entry, times m: the antiderivatives (Section
    # 2.1) grow with the corner coordinates, which reach m M / 2 cells, so the
    # rounding of their four-corner difference grows with m (the oracle itself
    # is long double)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-14 * m * scale)


@pytest.mark.parametrize("quantity", ["force", "potential"])
@pytest.mark.parametrize("M,kind,m,kx,ky,aspect", [(16, 1, 1, 0, 0, 0.5), (32, 2, 2, 1, 0, 2.5),
                                                   (16, 3, 3, 2, 1, 0.3), (32, 3, 4, 0, 3, 1.7)])
def test_kernel_table_rectangular_cells(ctx, M, kind, m, kx, ky, aspect, quantity):
    """Tables of cells of height aspect x width (v in units of the width)."""
    got = ctx.kernel_table(M, kind, m, kx, ky, quantity=quantity, aspect=aspect)
    want = np.zeros_like(got)
    for ny in range(M):
        for nx in range(M):
            if nx == M // 2 or ny == M // 2:
                continue
            sx = nx if nx < M // 2 else nx - M
            sy = ny if ny < M // 2 else ny - M
            if kind == 1:
                ua, va, w = -sx - 0.5, -sy - 0.5, 1.0
            elif kind == 2:
                ua, va, w = -m * sx + kx - m / 2, -m * sy + ky - m / 2, 1.0
            else:
                ua, va, w = -m * sx - kx - 0.5, -m * sy - ky - 0.5, float(m)
            va *= aspect
            if quantity == "force":
                c = oracle.cell_integrals(ua, ua + w, va, va + w * aspect)
                if kind == 3:
                    c[[1, 2, 4, 5]] /= m
                want[:, ny, nx] = c
            else:
                c = oracle.cell_potential_integrals(ua, ua + w, va, va + w * aspect)
                if kind == 3:
                    c = c / np.array([m, m * m, m * m])
                want[:3, ny, nx] = c
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-14 * m * max(aspect, 1) * scale)


# ---------------------------------------------------------------------------
# whole solves, full field
# ---------------------------------------------------------------------------

def H(levels, ratio=2, n0=None, x0=-1.0, y0=-1.0, aspect=1.0):
    n0 = n0 or levels[0][0]
    return synth.nested_hierarchy(x0, y0, 2.0 / n0, ratio, levels, aspect)


HIERS = {
    "1x1": H([(1, 0, 0)]),
    "1x5": H([(5, 0, 0)]),
    "1x37": H([(37, 0, 0)]),
    "1x64": H([(64, 0, 0)]),
    "2lev_20_12": H([(20, 0, 0), (12, 10, 16)]),
    "2lev_centred_32": H([(32, 0, 0), (32, 16, 16)]),
    "2lev_tiny_child": H([(9, 0, 0), (2, 4, 14)]),
    "3lev_ragged": H([(24, 0, 0), (18, 8, 20), (10, 30, 48)]),
    "3lev_corner": H([(16, 0, 0), (16, 16, 0), (8, 56, 0)]),
    "ratio4_2lev": H([(16, 0, 0), (16, 16, 24)], ratio=4),
    "ratio4_3lev": H([(12, 0, 0), (16, 12, 8), (8, 80, 44)], ratio=4),
    "4lev": H([(16, 0, 0), (16, 8, 8), (16, 24, 20), (8, 60, 52)]),
    # m = 16 pair whose target spans more columns than 2M of the coarse lattice
    "ratio4_deep": H([(6, 0, 0), (20, 4, 4), (44, 44, 44)], ratio=4),
    # odd ratio (m = 3, 9)
    "ratio3_2lev": H([(18, 0, 0), (15, 12, 21)], ratio=3),
    "ratio3_3lev": H([(12, 0, 0), (18, 9, 6), (27, 36, 30)], ratio=3),
    # five levels (m up to 16 through ratio 2: 256 Case-2 phases of one row)
    "5lev": H([(16, 0, 0), (16, 8, 8), (16, 24, 24), (16, 56, 56), (16, 120, 120)]),
    # rectangular cells (height = aspect x width)
    "aspect_0p5_3lev": H([(20, 0, 0), (16, 10, 8), (12, 26, 22)], aspect=0.5, y0=-0.5),
    "aspect_2p5_ratio3": H([(12, 0, 0), (18, 9, 6)], ratio=3, aspect=2.5, y0=-2.5),
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(HIERS))
def test_full_field_parity(ctx, name, dtype):
    hier = HIERS[name]
    sig, dx, dy = rand_fields(hier, seed=name_seed(name))
    ox, oy = oracle.forces(hier, sig, dx, dy)
    gx, gy = gpu_solve(ctx, hier, sig, dx, dy, dtype)
    err = rel_l2_full(hier, gx, gy, ox, oy)
    print(f"{name} {dtype} rel-L2 {err:.3e}")
    assert err <= TOL[dtype]
    assert covered_are_zero(hier, gx, gy)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(HIERS))
def test_estimated_slopes_parity(ctx, name, dtype):
    """TD_SLOPES_ESTIMATE (slopes from sigma inside the solve) against the
    oracle's estimate fed to the oracle's direct sum.  Random sigma in every
    cell, covered cells included (their values enter their neighbours'
    slopes); patches one and two cells wide take the degenerate branches."""
    hier = HIERS[name]
    sig, _, _ = rand_fields(hier, seed=name_seed(name) + 1, slopes=False)
    dx, dy = oracle.slopes(hier, sig)
    ox, oy = oracle.forces(hier, sig, dx, dy)
    gx, gy = gpu_solve(ctx, hier, sig, None, None, dtype, slopes="estimate")
    if max(np.abs(a).max() for a in ox + oy) == 0:
        # one cell, slope 0: the cell's force on itself vanishes by symmetry
        assert max(np.abs(a).max() for a in gx + gy) <= 1e-12 * np.abs(sig[0]).max()
        return
    err = rel_l2_full(hier, gx, gy, ox, oy)
    print(f"{name} {dtype} estimated slopes rel-L2 {err:.3e}")
    assert err <= TOL[dtype]
    assert covered_are_zero(hier, gx, gy)


def test_estimated_slopes_request_errors(ctx):
    """Slopes passed together with TD_SLOPES_ESTIMATE, an unknown mode, or a
    field pointer not aligned to the element size: TD_EINVAL, nothing
    launched."""
    import ctypes
    import torch
    from paper_1603_03142_amd import _binding as B
    hier = HIERS["2lev_20_12"]
    plan = ctx.plan(hier, "f64")
    sig = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in hier.patches]
    fx, fy = plan.outputs()
    for dsdx, mode in ((sig, B.TD_SLOPES_ESTIMATE), (None, 7), (None, -1)):
        req = B.make_request(plan.handle, sig, dsdx, None, fx, fy, mode)
        assert B.lib().td_solve(ctypes.byref(req), None) == B.TD_EINVAL
    flat = torch.zeros(sum(p.n * p.n for p in hier.patches) + 1, dtype=torch.float64,
                       device="cuda")
    odd = [flat, flat]
    req = B.make_request(plan.handle, odd, None, None, fx, fy, B.TD_SLOPES_GIVEN)
    ptrs = (ctypes.c_void_p * 2)(flat.data_ptr() + 4, flat.data_ptr())
    req.sigma = ctypes.cast(ptrs, B.VPP)
    assert B.lib().td_solve(ctypes.byref(req), None) == B.TD_EINVAL
    assert b"aligned" in B.lib().td_last_error()
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_no_slopes(ctx, dtype):
    hier = HIERS["3lev_ragged"]
    sig, _, _ = rand_fields(hier, seed=11, slopes=False)
    ox, oy = oracle.forces(hier, sig)
    gx, gy = gpu_solve(ctx, hier, sig, None, None, dtype)
    assert rel_l2_full(hier, gx, gy, ox, oy) <= TOL[dtype]


def test_config1_maclaurin(ctx):
    """64x64 level, Maclaurin disk R = 0.8, FP64: whole field vs the oracle."""
    hier, fn = synth.config1()
    sig, dx, dy = synth.sample_fields(hier, fn, "central")
    ox, oy = oracle.forces(hier, sig, dx, dy)
    gx, gy = gpu_solve(ctx, hier, sig, dx, dy, "f64")
    err = rel_l2_full(hier, gx, gy, ox, oy)
    print(f"config1 f64 rel-L2 {err:.3e}")
    assert err <= 1e-12


def test_determinism(ctx):
    hier = HIERS["3lev_ragged"]
    sig, dx, dy = rand_fields(hier, seed=5)
    plan = ctx.plan(hier, "f32")
    a = gpu_solve(ctx, hier, sig, dx, dy, "f32", plan)
    b = gpu_solve(ctx, hier, sig, dx, dy, "f32", plan)
    for k in range(len(hier.patches)):
        assert np.array_equal(a[0][k], b[0][k]) and np.array_equal(a[1][k], b[1][k])
