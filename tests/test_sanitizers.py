"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle/direct_sum.c), built with gcc and both sanitizers (any
  report aborts), solves small nested and multi-patch hierarchies, the
  generalized convolutions of Section 2.2 and two cell integrals; its output
  must equal the regular oracle build's.
* The C ABI's host-only logic (hierarchy checks, host-only planning with its
  job-list bounds proof: td_hierarchy_check, td_plan_check), built host-only
  with both sanitizers and stub device launchers, runs on valid and invalid
  random hierarchies; statuses and workspace sizes must equal the regular
  library's.

Sanitizers apply to host code only (the device code is not compiled here).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")


def _hierarchies():
    out = [
        synth.nested_hierarchy(-1.0, -1.0, 2.0 / 8, 2, [(8, 0, 0), (8, 4, 4)]),
        synth.nested_hierarchy(-1.0, -1.0, 2.0 / 9, 3, [(9, 0, 0), (6, 6, 9)]),
        synth.random_patches(5, n0=8, levels=3, per_level=2),
    ]
    h = synth.nested_hierarchy(-1.0, -1.0, 2.0 / 10, 2, [(10, 0, 0), (8, 6, 2)])
    h.aspect = 0.5
    out.append(h)
    return out


@pytest.fixture(scope="module")
def oracle_san(tmp_path_factory):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("san") / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off",
                           "-o", exe, os.path.join(ROOT, "oracle", "direct_sum.c"),
                           os.path.join(SAN, "oracle_driver.c"), "-lm"])
    return exe


@pytest.mark.parametrize("case", range(4))
def test_oracle_under_sanitizers(oracle_san, case):
    hier = _hierarchies()[case]
    rng = np.random.Generator(np.random.PCG64(100 + case))
    fields = [[rng.normal(size=(p.n, p.n)) for p in hier.patches] for _ in range(3)]
    lines = [f"{len(hier.patches)} {hier.x0!r} {hier.y0!r} {hier.h0!r} {hier.aspect!r} {hier.ratio}"]
    lines += [f"{p.level} {p.n} {p.ox} {p.oy}" for p in hier.patches]
    for k in range(len(hier.patches)):
        for f in fields:
            lines.append(" ".join(repr(float(v)) for v in f[k].ravel()))
    tp = np.concatenate([np.full(p.n * p.n, k) for k, p in enumerate(hier.patches)])
    ti = np.concatenate([np.tile(np.arange(p.n), p.n) for p in hier.patches])
    tj = np.concatenate([np.repeat(np.arange(p.n), p.n) for p in hier.patches])
    lines.append(str(len(tp)))
    lines += [f"{a} {b} {c}" for a, b, c in zip(tp, ti, tj)]
    r = subprocess.run([oracle_san], input="\n".join(lines) + "\n", capture_output=True,
                       text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    rows = [list(map(float, l.split())) for l in r.stdout.strip().split("\n")]
    got = np.array(rows[:len(tp)])
    fx, fy = oracle.forces(hier, *fields, targets=(tp, ti, tj))
    phi = oracle.potential(hier, *fields, targets=(tp, ti, tj))
    np.testing.assert_allclose(got[:, 0], fx, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got[:, 1], fy, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got[:, 2], phi, rtol=1e-13, atol=1e-15)
    b = np.arange(1.0, 9.0)
    c = np.array([1.0, -1.0, 2.0, -2.0])
    for mode in (1, 2, 3):
        np.testing.assert_allclose(rows[len(tp) + mode - 1], oracle.genconv1d(mode, 2, b, c, 12))
    want = list(oracle.cell_integrals(0.0, 1.0, 1.0, 2.0)) + \
        list(oracle.cell_potential_integrals(-3.0, -2.0, -0.5, 0.5))
    np.testing.assert_allclose(rows[len(tp) + 3], want, rtol=1e-15)


def _abi_san(tmp):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = os.path.join(tmp, "abi_san")
    csrc = os.path.join(ROOT, "paper_1603_03142_amd", "csrc")
    # host-only compilation: the sanitizers instrument host code only
    cmd = [hipcc, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "--offload-host-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-x", "hip", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "td_api.cpp"), os.path.join(SAN, "launch_stubs.cpp"),
           "-x", "c++", os.path.join(SAN, "abi_driver.cpp"), "-o", exe]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return exe


def _random_hierarchies(count=150):
    rng = np.random.Generator(np.random.PCG64(77))
    out = []
    for k in range(count):
        if k % 3 == 0:
            h = synth.random_patches(int(rng.integers(0, 10 ** 6)), n0=int(rng.choice([8, 16, 32])),
                                     levels=int(rng.integers(1, 4)),
                                     per_level=int(rng.integers(1, 3)),
                                     ratio=int(rng.choice([2, 3, 4])))
        else:
            h = synth._random_nested(rng, int(rng.choice([16, 32, 64, 128])), int(rng.integers(1, 5)))
        pats = [(p.level, p.n, p.ox, p.oy) for p in h.patches]
        if k % 5 == 4 and len(pats) > 1:  # break it: off the parent lattice, or outside
            lv, n, ox, oy = pats[-1]
            pats[-1] = (lv, n, ox + (1 if k % 2 else 10 ** 5), oy)
        out.append((h.x0, h.y0, h.h0, h.ratio, getattr(h, "aspect", 1.0), pats))
    return out


def test_abi_host_logic_under_sanitizers(tmp_path):
    import ctypes
    from paper_1603_03142_amd import _binding as B
    exe = _abi_san(str(tmp_path))
    hs = _random_hierarchies()
    text = "\n".join(f"{x0!r} {y0!r} {h0!r} {r} {a!r} {len(p)} " +
                     " ".join(f"{l} {n} {ox} {oy}" for l, n, ox, oy in p)
                     for x0, y0, h0, r, a, p in hs) + "\n"
    res = subprocess.run([exe], input=text, capture_output=True, text=True, env=ENV, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-3000:]
    got = [tuple(map(int, l.split())) for l in res.stdout.strip().split("\n")]
    assert len(got) == len(hs)
    lib = B.lib()
    bad = 0
    for (x0, y0, h0, r, a, p), g in zip(hs, got):
        arr = (B.td_patch * len(p))(*[B.td_patch(*q) for q in p])
        h = B.td_hierarchy(x0, y0, h0, r, len(p), ctypes.cast(arr, ctypes.POINTER(B.td_patch)), a)
        chk = lib.td_hierarchy_check(ctypes.byref(h))
        w32, w64 = ctypes.c_size_t(), ctypes.c_size_t()
        s32 = lib.td_plan_check(ctypes.byref(h), B.TD_F32, ctypes.byref(w32))
        s64 = lib.td_plan_check(ctypes.byref(h), B.TD_F64, ctypes.byref(w64))
        assert g == (chk, s32, w32.value if s32 == 0 else g[2], s64, w64.value if s64 == 0 else g[4])
        bad += chk != 0
    assert 0 < bad < len(hs)  # both valid and invalid hierarchies were exercised
