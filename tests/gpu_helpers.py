"""Shared helpers of the GPU parity tests: seeded inputs from ``synth``,
solves through the C ABI, comparison with the oracle."""
import math
import zlib

import numpy as np

import oracle
import synth


def name_seed(name: str) -> int:
    """A seed fixed by a case name (the built-in str hash varies per process)."""
    return zlib.crc32(name.encode()) % 1000


def rand_fields(hier, seed, slopes=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    sig = [rng.normal(size=(p.n, p.n)) for p in hier.patches]
    if not slopes:
        return sig, None, None
    dx = [rng.normal(size=(p.n, p.n)) for p in hier.patches]
    dy = [rng.normal(size=(p.n, p.n)) for p in hier.patches]
    return sig, dx, dy


def to_dev(arrs, dtype):
    import torch
    if arrs is None:
        return None
    return [torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda") if a is not None
            else None for a in arrs]


def gpu_solve(ctx, hier, sig, dx, dy, dtype="f64", plan=None, slopes="given"):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    if plan is None:
        plan = ctx.plan(hier, dtype)
    fx, fy = plan.solve(to_dev(sig, td), to_dev(dx, td), to_dev(dy, td), slopes=slopes)
    torch.cuda.synchronize()
    return [a.double().cpu().numpy() for a in fx], [a.double().cpu().numpy() for a in fy]


def active_masks(hier):
    return [~synth.covered_mask(hier, p) for p in hier.patches]


def rel_l2_full(hier, gx, gy, ox, oy):
    num = den = 0.0
    for k, act in enumerate(active_masks(hier)):
        num += ((gx[k] - ox[k])[act] ** 2).sum() + ((gy[k] - oy[k])[act] ** 2).sum()
        den += (ox[k][act] ** 2).sum() + (oy[k][act] ** 2).sum()
    return math.sqrt(num / den)


def covered_are_zero(hier, gx, gy):
    for k, act in enumerate(active_masks(hier)):
        if not (np.all(gx[k][~act] == 0) and np.all(gy[k][~act] == 0)):
            return False
    return True


def sampled(hier, gx, gy, targets):
    tp, ti, tj = targets
    return (np.array([gx[p][j, i] for p, i, j in zip(tp, ti, tj)]),
            np.array([gy[p][j, i] for p, i, j in zip(tp, ti, tj)]))


def rel_l2(ax, ay, bx, by):
    return math.sqrt((((ax - bx) ** 2).sum() + ((ay - by) ** 2).sum()) /
                     ((bx ** 2).sum() + (by ** 2).sum()))


def level_rel_l2(hier, targets, gx, gy, ox, oy):
    """rel-L2 of sampled values per level of the hierarchy ({level: err}),
    each over the targets on that level's patches; gx, gy, ox, oy are flat
    arrays aligned with ``targets``."""
    tp = np.asarray(targets[0])
    lev = np.array([hier.patches[p].level for p in tp])
    out = {}
    for l in sorted(set(lev.tolist())):
        s = lev == l
        out[l] = rel_l2(gx[s], gy[s], ox[s], oy[s])
    return out


def report(name, hier, targets, gx, gy, ox, oy):
    """Overall rel-L2, per-level rel-L2 and the largest absolute error of a
    sampled comparison, printed for the log and returned."""
    err = rel_l2(gx, gy, ox, oy)
    per = level_rel_l2(hier, targets, gx, gy, ox, oy)
    amax = float(max(np.abs(gx - ox).max(), np.abs(gy - oy).max()))
    print(f"{name}: rel-L2 {err:.3e}, per level "
          + ", ".join(f"{l}: {e:.3e}" for l, e in per.items())
          + f", max abs {amax:.3e} ({len(gx)} targets)", flush=True)
    return err, per, amax
