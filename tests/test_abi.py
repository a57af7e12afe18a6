"""The C-ABI library loads and exports every entry point its header declares;
host-only logic (hierarchy validation and snapping) checked without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thindisk.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(td_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    assert "td_solve" in names and "td_plan_create" in names and "td_server_submit" in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    from paper_1603_03142_amd import _binding
    L = _binding.lib()
    for name in declared():
        assert hasattr(L, name), name
    assert sorted(_binding.EXPORTS) == declared()
    assert b"gfx950" in L.td_version()


def test_binding_structs_match_header(tmp_path):
    """The ctypes structs and constants of the binding have the header's
    layout and values (a C probe compiled against the header with gcc)."""
    from paper_1603_03142_amd import _binding as B
    probe = tmp_path / "probe.c"
    probe.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "thindisk.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %d %d %d %d\\n", sizeof(td_patch), sizeof(td_hierarchy),'
        " offsetof(td_hierarchy, patches), sizeof(td_request), offsetof(td_request, fy),"
        " offsetof(td_request, slopes), TD_SLOPES_GIVEN, TD_SLOPES_ESTIMATE, TD_MAX_PATCHES,"
        " TD_MAX_LEVELS);\n"
        '  printf("%zu\\n", offsetof(td_hierarchy, aspect));\n'
        '  printf("%d %d\\n", TD_FORCE, TD_POTENTIAL);\n  return 0;\n}\n')
    exe = tmp_path / "probe"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(probe), "-o",
                    str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(B.td_patch), ctypes.sizeof(B.td_hierarchy), B.td_hierarchy.patches.offset,
            ctypes.sizeof(B.td_request), B.td_request.fy.offset, B.td_request.slopes.offset,
            B.TD_SLOPES_GIVEN, B.TD_SLOPES_ESTIMATE, B.TD_MAX_PATCHES, B.TD_MAX_LEVELS,
            B.td_hierarchy.aspect.offset, B.TD_FORCE, B.TD_POTENTIAL]
    assert got == want


def _check(levels, ratio=2, h0=2 / 16, patches=None, aspect=0.0):
    """levels: one (n, ox, oy) patch per level; patches: (level, n, ox, oy)."""
    from paper_1603_03142_amd import _binding as B
    pats = patches if patches is not None else [(l, *lv) for l, lv in enumerate(levels)]
    arr = (B.td_patch * len(pats))(*[B.td_patch(*p) for p in pats])
    h = B.td_hierarchy(-1.0, -1.0, h0, ratio, len(pats), ctypes.cast(arr, ctypes.POINTER(B.td_patch)),
                       aspect)
    return B.lib().td_hierarchy_check(ctypes.byref(h))


def test_hierarchy_validation_codes():
    from paper_1603_03142_amd import _binding as B
    assert _check([(16, 0, 0)]) == B.TD_OK
    assert _check([(16, 0, 0), (16, 8, 8)]) == B.TD_OK
    assert _check([(16, 0, 0), (16, 8, 8), (8, 20, 22)]) == B.TD_OK
    assert _check([(16, 0, 0), (16, 7, 8)]) == B.TD_EALIGN          # odd offset
    assert _check([(16, 0, 0), (15, 8, 8)]) == B.TD_EALIGN          # odd width
    assert _check([(16, 0, 0), (16, 18, 8)]) == B.TD_ENEST          # sticks out
    assert _check([(16, 0, 0), (34, 0, 0)]) == B.TD_ENEST           # wider than parent
    assert _check([(16, 2, 0)]) == B.TD_EINVAL                      # level-0 offset
    assert _check([(16, 0, 0)], ratio=5) == B.TD_EUNSUPPORTED
    # rectangular cells: aspect 0 (square) or in [1/64, 64]
    assert _check([(16, 0, 0), (8, 4, 4)], aspect=0.5) == B.TD_OK
    assert _check([(16, 0, 0)], aspect=64.0) == B.TD_OK
    for bad in (-1.0, 100.0, 1e-3, float("nan"), float("inf")):
        assert _check([(16, 0, 0)], aspect=bad) == B.TD_EINVAL, bad
    assert _check([(18, 0, 0), (15, 12, 21)], ratio=3) == B.TD_OK
    assert _check([(18, 0, 0), (15, 12, 20)], ratio=3) == B.TD_EALIGN       # off the lattice
    assert _check([(9, 0, 0), (9, 3, 3), (9, 9, 9), (9, 27, 27)], ratio=3) == B.TD_EUNSUPPORTED  # 27x
    assert _check([(0, 0, 0)]) == B.TD_EINVAL
    assert _check([(2048, 0, 0)]) == B.TD_OK
    assert _check([(2049, 0, 0)]) == B.TD_EINVAL                    # beyond TD_MAX_N
    assert _check([(16, 0, 0), (16, 56, 8)], ratio=4) == B.TD_ENEST
    assert _check([(16, 0, 0), (16, 16, 24)], ratio=4) == B.TD_OK
    assert _check([(8, 0, 0)] * 9) == B.TD_EINVAL                   # too many patches
    assert "npatches" in B.lib().td_last_error().decode()
    # several patches per level
    two = [(0, 16, 0, 0), (1, 8, 4, 12), (1, 8, 20, 12)]
    assert _check(None, patches=two) == B.TD_OK
    assert _check(None, patches=[(0, 16, 0, 0), (1, 8, 4, 12), (1, 8, 10, 12)]) == B.TD_EINVAL  # overlap
    assert "overlaps" in B.lib().td_last_error().decode()
    assert _check(None, patches=[(0, 16, 0, 0), (1, 8, 4, 12), (1, 8, 28, 12)]) == B.TD_ENEST   # outside
    assert _check(None, patches=[(0, 16, 0, 0), (1, 8, 4, 12), (0, 8, 0, 0)]) == B.TD_EINVAL    # order
    assert _check(None, patches=[(0, 16, 0, 0), (2, 8, 4, 12)]) == B.TD_EINVAL                  # level gap
    # a level-2 patch inside the second level-1 patch only
    three = two + [(2, 8, 44, 28)]
    assert _check(None, patches=three) == B.TD_OK
    assert _check(None, patches=two + [(2, 8, 30, 28)]) == B.TD_ENEST  # straddles both


def test_snap_matches_python_generator():
    """td_hierarchy_snap and synth.snap_offsets implement the same rounding."""
    import synth
    from paper_1603_03142_amd import _binding as B
    h0 = 2.0 / 512
    want = synth.snap_offsets(-1.0, -1.0, h0, 2, [512] * 4, [(0.3, 0.0)] * 3)
    lv = (B.td_patch * 4)(*[B.td_patch(l, 512, 0, 0) for l in range(4)])
    h = B.td_hierarchy(-1.0, -1.0, h0, 2, 4, ctypes.cast(lv, ctypes.POINTER(B.td_patch)))
    cx = (ctypes.c_double * 3)(0.3, 0.3, 0.3)
    cy = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    assert B.lib().td_hierarchy_snap(ctypes.byref(h), lv, cx, cy) == B.TD_OK
    got = [(lv[i].n, lv[i].ox, lv[i].oy) for i in range(4)]
    assert got == want == [(512, 0, 0), (512, 410, 256), (512, 1076, 768), (512, 2406, 1792)]
    assert B.lib().td_hierarchy_check(ctypes.byref(h)) == B.TD_OK


def test_status_strings():
    from paper_1603_03142_amd import _binding as B
    for k, name in B._STATUS.items():
        assert B.lib().td_status_string(k).decode() == name


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    from paper_1603_03142_amd import _binding as B
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError):
        B.lib()


def _random_hierarchy(rng):
    import synth
    ratio = int(rng.choice([2, 4]))
    nlev = int(rng.integers(1, 5 if ratio == 2 else 4))
    n0 = int(rng.integers(1, 70))
    lv = [(n0, 0, 0)]
    for _ in range(1, nlev):
        pn, pox, poy = lv[-1]
        if pn < 1:
            break
        w = int(rng.integers(1, pn + 1))          # parent cells covered
        n = w * ratio
        if n > 2048:
            break
        kx = int(rng.integers(0, pn - w + 1))
        ky = int(rng.integers(0, pn - w + 1))
        lv.append((n, ratio * (pox + kx), ratio * (poy + ky)))
    return synth.nested_hierarchy(-1.0, -1.0, 2.0 / n0, ratio, lv)


def test_plan_check_random_hierarchies():
    """Host-side proof of every job's bounds and row coverage on random
    nested hierarchies (ragged sizes, ratios 2 and 4, 1-4 levels)."""
    import numpy as np
    import paper_1603_03142_amd as td
    rng = np.random.default_rng(12)
    for _ in range(150):
        h = _random_hierarchy(rng)
        for dt in ("f32", "f64"):
            assert td.check_plan(h, dt) > 0


def test_plan_check_workloads():
    import paper_1603_03142_amd as td
    import synth
    for f in (synth.config1, synth.config2, synth.config3):
        h, _ = f()
        assert td.check_plan(h, "f32") > 0
    for h, _ in synth.config4(count=16):
        assert td.check_plan(h, "f32") > 0
    # band-limited column inputs (phase sub-grids of at most M/16 rows on
    # M = 1024, M/32 on M = 2048): the band test's hierarchy and a
    # five-level 1024^2 request (m = 16)
    import numpy as np
    from test_gpu_band import band_hierarchy
    five = synth._random_nested(np.random.Generator(np.random.PCG64(55)), 1024, 5)
    for h in (band_hierarchy(264), band_hierarchy(520), five):
        for dt in ("f32", "f64"):
            assert td.check_plan(h, dt) > 0


def test_plan_check_random_patches():
    """The same host-side proof on hierarchies with several patches per
    level (ratios 2 and 4, up to 4 levels, at most 8 patches)."""
    import paper_1603_03142_amd as td
    import synth
    multi = 0
    for seed in range(120):
        h = synth.random_patches(seed, n0=[16, 24, 36, 40][seed % 4], levels=2 + seed % 3,
                                 per_level=1 + seed % 3, ratio=[2, 4, 3][seed % 3])
        multi += any(sum(p.level == l for p in h.patches) > 1 for l in range(4))
        for dt in ("f32", "f64"):
            assert td.check_plan(h, dt) > 0
    assert multi > 50
    for ex, n in ((3, 32), (3, 1024), (4, 64), (4, 512)):
        assert td.check_plan(synth.example_hierarchy(ex, n), "f32") > 0


def test_entry_points_refuse_null_handles():
    """Host-side argument checks of the batch, server, debug and
    allocation-free entry points: NULL handles and unknown modes are refused
    with TD_EINVAL before anything touches a device."""
    from paper_1603_03142_amd import _binding as B
    lib = B.lib()
    count = ctypes.c_uint64(7)
    assert lib.td_batch_set_launch(None, B.TD_LAUNCH_DIRECT) == B.TD_EINVAL
    assert lib.td_context_set_debug(None, B.TD_DEBUG_NONFINITE) == B.TD_EINVAL
    assert lib.td_debug_nonfinite(None, ctypes.byref(count)) == B.TD_EINVAL
    assert lib.td_solve_noalloc(None, None) == B.TD_EINVAL
    req = B.td_request()
    assert lib.td_solve_noalloc(ctypes.byref(req), None) == B.TD_EINVAL  # no plan
    assert lib.td_server_stats2(None, None, None) == B.TD_EINVAL
    assert lib.td_batch_solve(None, None, 0, None) == B.TD_EINVAL
    assert "NULL" in lib.td_last_error().decode()
