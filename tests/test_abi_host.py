"""CPU tests of the C ABI library: it loads, exports every declared entry point, rejects
misuse without a GPU, and its host build of the device exp matches the oracle."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "safegpu.h")


@pytest.fixture(scope="module")
def lib():
    import paper_1410_6685_amd as sg
    if not os.path.exists(sg.LIB_PATH):
        from paper_1410_6685_amd import build
        build.build(verbose=False)
    return sg


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:sg_status|const char\*)\s+(sg_\w+)\(", text, re.M)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    assert len(syms) >= 50
    for s in ("sg_ctx_create", "sg_map", "sg_filter", "sg_program_execute", "sg_batch_create", "sg_matmul"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (sg_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    L = lib.load()
    for s in declared_symbols():
        assert hasattr(L, s)


def test_misuse_is_rejected_without_gpu(lib):
    from ctypes import byref, c_void_p
    L = lib.load()
    h = c_void_p()
    assert L.sg_fn_unary(99, byref(h)) == 1
    assert L.sg_pred_cmp(42, 0.0, byref(h)) == 1
    assert L.sg_map(None, None, byref(h)) == 1
    assert L.sg_program_execute(None, None, 0, None) == 1
    assert L.sg_fn_affine(2.0, 1.0, byref(h)) == 0
    f = h.value
    g = c_void_p()
    assert L.sg_fn_compose(f, f, byref(g)) == 0
    assert L.sg_fn_release(g) == 0 and L.sg_fn_release(f) == 0
    # no device here: creating a context reports a device error instead of crashing
    ctx = c_void_p()
    st = L.sg_ctx_create(0, None, byref(ctx))
    assert st in (0, 5)
    if st == 0:
        L.sg_ctx_destroy(ctx)


def test_device_exp_on_host_matches_oracle(lib):
    t = W.uniform_f32(1 << 22, 99, -104.0, 89.0)
    got, slow = lib.host_exp_rn(t)
    ref, hard = oracle.exp_rn32(t, return_hard=True)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    got_h, _ = lib.host_exp_rn(t[hard])
    assert np.array_equal(got_h.view(np.uint32), ref[hard].view(np.uint32))
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 88.72283935546875, 88.72283172607422,
                        -103.97208404541016, -103.97207641601562, -87.33654022216797, 1e-30], np.float32)
    got, _ = lib.host_exp_rn(special)
    ref = oracle.exp_rn32(special)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok].view(np.uint32), ref[ok].view(np.uint32))


def test_device_exp_slow_path_cases(lib):
    """Collect inputs that take the double-double path and check them one by one."""
    t = W.uniform_f32(1 << 23, 123, -104.0, 0.0)
    got, slow = lib.host_exp_rn(t)
    assert slow > 0
    # find them: recompute in blocks and keep blocks that report slow elements
    idx = []
    for b in range(0, t.size, 1 << 16):
        _, s = lib.host_exp_rn(t[b:b + (1 << 16)])
        if s:
            for i in range(b, min(b + (1 << 16), t.size)):
                if lib.host_exp_rn(t[i:i + 1])[1]:
                    idx.append(i)
    assert len(idx) == slow
    ref = oracle.exp_rn32(t[idx])
    assert np.array_equal(got[idx].view(np.uint32), ref.view(np.uint32))


def test_device_exp_fast_path_sweep(tmp_path):
    """The fast path of the device exp agrees with its double-double path wherever it does not
    flag a hard case (every 61st binary32 argument of the finite, nonzero range; the same
    program with stride 1 is the exhaustive sweep)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "exp_sweep")
    subprocess.run([gxx, "-O2", "-std=c++20", "-ffp-contract=off", "-pthread", os.path.join(here, "exp_sweep.cpp"),
                    "-o", exe], check=True)
    r = subprocess.run([exe, "61", "8"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    total, hard, bad = (int(v) for v in r.stdout.split()[1::2])
    assert bad == 0 and total > 36_000_000 and hard < total // 500
