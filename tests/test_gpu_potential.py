"""The potential (eq. eqnPhixy0: Green's function -1/rho, G = 1) through the
C ABI: potential plans (TD_POTENTIAL) against the oracle's direct sum, their
kernel tables against the oracle's cell integrals, force and potential plans
in one batch, and second-order convergence to the appendix's analytic
potential.  Tolerances as for the force: FP64 1e-12, FP32 1e-5 rel-L2 over
active cells; covered cells exactly 0."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import name_seed, rand_fields, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import paper_1603_03142_amd as td
    c = td.Context(0)
    yield c
    c.close()


def H(levels, ratio=2, n0=None, aspect=1.0):
    n0 = n0 or levels[0][0]
    return synth.nested_hierarchy(-1.0, -1.0, 2.0 / n0, ratio, levels, aspect)


HIERS = {
    "1x1": H([(1, 0, 0)]),
    "1x37": H([(37, 0, 0)]),
    "2lev_20_12": H([(20, 0, 0), (12, 10, 16)]),
    "2lev_tiny_child": H([(9, 0, 0), (2, 4, 14)]),
    "3lev_ragged": H([(24, 0, 0), (18, 8, 20), (10, 30, 48)]),
    "4lev": H([(16, 0, 0), (16, 8, 8), (16, 24, 20), (8, 60, 52)]),
    "ratio3_3lev": H([(12, 0, 0), (18, 9, 6), (27, 36, 30)], ratio=3),
    "ratio4_deep": H([(6, 0, 0), (20, 4, 4), (44, 44, 44)], ratio=4),
    "aspect_0p6": H([(24, 0, 0), (18, 8, 20), (10, 30, 48)], aspect=0.6),
}


def gpu_potential(ctx, hier, sig, dx, dy, dtype, slopes="given"):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    plan = ctx.plan(hier, dtype, quantity="potential")
    phi, none = plan.solve(to_dev(sig, td), to_dev(dx, td), to_dev(dy, td), slopes=slopes)
    torch.cuda.synchronize()
    assert none is None
    return [a.double().cpu().numpy() for a in phi]


def rel_l2_phi(hier, got, want):
    num = den = 0.0
    for k, p in enumerate(hier.patches):
        act = ~synth.covered_mask(hier, p)
        num += ((got[k] - want[k])[act] ** 2).sum()
        den += (want[k][act] ** 2).sum()
        assert np.all(got[k][~act] == 0)
    return math.sqrt(num / den)


TABLE_CASES = [(16, 1, 1, 0, 0), (32, 1, 1, 0, 0), (16, 2, 2, 1, 0), (32, 2, 4, 1, 3),
               (16, 3, 2, 0, 1), (32, 3, 4, 3, 2), (16, 2, 3, 1, 1), (32, 3, 9, 4, 8)]


@pytest.mark.parametrize("M,kind,m,kx,ky", TABLE_CASES)
def test_potential_kernel_table_vs_oracle(ctx, M, kind, m, kx, ky):
    got = ctx.kernel_table(M, kind, m, kx, ky, quantity="potential")
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
            c = oracle.cell_potential_integrals(ua, ua + w, va, va + w)
            if kind == 3:
                c = c / np.array([m, m * m, m * m])
            want[:3, ny, nx] = c
    assert np.all(got[3:] == 0)
    scale = np.abs(want).max()
    # corner differences of antiderivatives that grow with the offset
    # (up to m M / 2 cells): a few ulp of the largest entry, times m
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-14 * m * scale)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("name", sorted(HIERS))
def test_potential_full_field_parity(ctx, name, dtype):
    hier = HIERS[name]
    sig, dx, dy = rand_fields(hier, seed=name_seed(name) + 7)
    want = oracle.potential(hier, sig, dx, dy)
    got = gpu_potential(ctx, hier, sig, dx, dy, dtype)
    err = rel_l2_phi(hier, got, want)
    print(f"{name} {dtype} potential rel-L2 {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_potential_estimated_slopes_and_patches(ctx, dtype):
    """Slopes estimated from sigma, on random multi-patch hierarchies of
    ratios 2, 3 and 4."""
    for seed in (3, 4, 5, 8):
        hier = synth.random_patches(seed, n0=[16, 24, 36, 40][seed % 4], levels=2 + seed % 3,
                                    per_level=1 + seed % 3, ratio=[2, 4, 3][seed % 3])
        sig, _, _ = rand_fields(hier, 90 + seed, slopes=False)
        want = oracle.potential(hier, sig, *oracle.slopes(hier, sig))
        got = gpu_potential(ctx, hier, sig, None, None, dtype, slopes="estimate")
        assert rel_l2_phi(hier, got, want) <= TOL[dtype], seed


def test_force_and_potential_plans_share_a_batch(ctx):
    """One batch of force and potential plans (the kernel family travels
    with each column job): every member equals its own single solve bit for
    bit, the potential's second output untouched."""
    import torch
    import paper_1603_03142_amd as td
    hiers = [HIERS["3lev_ragged"], HIERS["2lev_20_12"], HIERS["ratio3_3lev"]]
    plans, fields = [], []
    for k, h in enumerate(hiers):
        for q in ("force", "potential"):
            plans.append(ctx.plan(h, "f32", quantity=q))
            sig, dx, dy = rand_fields(h, 300 + k)
            fields.append((to_dev(sig, torch.float32), to_dev(dx, torch.float32),
                           to_dev(dy, torch.float32)))
    single = [p.solve(*f) for p, f in zip(plans, fields)]
    torch.cuda.synchronize()
    res = td.Batch(ctx, plans).solve(fields)
    torch.cuda.synchronize()
    for p, (a0, a1), (b0, b1) in zip(plans, single, res):
        for x, y in zip(a0, b0):
            assert torch.equal(x, y)
        if p.quantity == "force":
            for x, y in zip(a1, b1):
                assert torch.equal(x, y)
        else:
            assert a1 is None and b1 is None


def test_potential_converges_to_the_appendix_pair(ctx):
    """sigma_{D5} (alpha = 0.85) on Example 1's grids, FP64, slopes from
    sigma: the mean error against the analytic potential falls about 4x per
    halving of h from N = 32 to 512 (no paper value to compare: the paper
    prints no potential errors)."""
    from scipy.interpolate import CubicSpline
    from oracle import analytic
    alpha = 0.85
    t = np.linspace(0.0, math.sqrt(1.45), 3001)
    r = t * t
    spl = CubicSpline(t, [float(analytic.potential(5, x, alpha)) for x in r])
    errs = []
    for n in (32, 64, 128, 256, 512):
        hier = synth.example_hierarchy(1, n)
        sig, _, _ = synth.sample_fields(hier, synth.disk_dn(5, alpha), "none")
        phi = gpu_potential(ctx, hier, sig, None, None, "f64", slopes="estimate")
        e = []
        for k, p in enumerate(hier.patches):
            X, Y = synth.cell_centres(hier, p)
            act = ~synth.covered_mask(hier, p)
            e.append(np.abs(phi[k][act] - spl(np.sqrt(np.hypot(X[act], Y[act])))))
        errs.append(np.concatenate(e).mean())
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    print("\npotential E1 vs analytic:", " ".join(f"{e:.4e}" for e in errs),
          " orders", " ".join(f"{o:.3f}" for o in orders))
    assert all(1.9 < o < 2.1 for o in orders)


@pytest.mark.parametrize("workload,count,dtype,tol", [
    ("two-level-256", 128, "f64", 1e-12), ("two-level-256", 128, "f32", 1e-5),
    ("four-level-512", 32, "f64", 1e-12), ("four-level-512", 32, "f32", 1e-5)])
def test_potential_full_size_sampled(ctx, workload, count, dtype, tol):
    """Potential plans at the benched sizes (sigma in, slopes estimated),
    sampled targets.  The potential weighs far cells more than the force
    (1/r against 1/r^2), where the tables' corner differences cancel most."""
    import bench
    hier, fn = bench.workload(workload)
    sig, _, _ = synth.sample_fields(hier, fn, "none")
    phi = gpu_potential(ctx, hier, sig, None, None, dtype, slopes="estimate")
    tg = synth.sample_targets(hier, count, seed=19)
    want = oracle.potential(hier, sig, *oracle.slopes(hier, sig), tg)
    got = np.array([phi[p][j, i] for p, i, j in zip(*tg)])
    err = math.sqrt(((got - want) ** 2).sum() / (want ** 2).sum())
    print(f"{workload} {dtype} potential sampled rel-L2 {err:.3e}")
    assert err <= tol
