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
    assert L.sg_ctx_set_plan_source(None, 1, None, 0, 3, None, None, 0.01) == 1
    assert L.sg_program_plan(None, None, None) == 1
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


def random_expression(g, depth=0):
    """A seeded expression of the agent grammar (mixed operators, literals, x, functions)."""
    r = g.integers(0, 10) if depth < 5 else g.integers(0, 3)
    if r == 0:
        return "x"
    if r == 1:
        return repr(float(np.float32(g.uniform(-4, 4))))[:8].rstrip("-.e") or "1"
    if r == 2:
        return f"{g.integers(0, 20)}.{g.integers(0, 100)}"
    if r == 3:
        return f"-{random_expression(g, depth + 1)}"
    if r == 4:
        return f"{['sqrt', 'abs', 'exp'][g.integers(0, 3)]}({random_expression(g, depth + 1)})"
    if r == 5:
        return f"({random_expression(g, depth + 1)})"
    return f"{random_expression(g, depth + 1)} {'+-*/'[g.integers(0, 4)]} {random_expression(g, depth + 1)}"


def test_expression_programs_match_oracle(lib):
    """The register programs the expression compiler gives a map (x and the result in one
    register, intermediate values in the free ones) compute the oracle's values bit for bit,
    with as many registers as the expression needs and with fewer (refused, never wrong)."""
    from oracle.expr import apply_expr, parse
    g = np.random.default_rng(12)
    x = np.concatenate([W.normal_f32(400, 2, 3.0), np.array([0, -0.0, 1, -1, 0.5, 1e-40, np.inf, -np.inf, np.nan],
                                                             np.float32)])
    fixed = ["x", "2", "-x", "x*x", "x - x*x", "(x+1)*(x-1)/(x*x+2)", "1/(1+exp(-x))", "((x+1)*(x+2))*((x+3)*(x+4))",
             "sqrt(abs(x)) - (x*0.25 - 1/(x+3))", "2 - (3 - (4 - x))", "(x*x+1)/((x+1)*(x-2) + (x*x)*(x+0.5))"]
    exprs = fixed + [random_expression(g) for _ in range(300)]
    refused = 0
    for src in exprs:
        try:
            parse(src)
        except ValueError:
            continue
        want = apply_expr(src, x)
        ok_once = False
        for regs in (1, 2, 3, 5, 8):
            try:
                got, nops = lib.host_expr_run(src, x, regs)
            except lib.SafeGPUError as e:
                assert e.status_name == "unsupported", (src, regs, e)
                refused += 1
                continue
            ok_once = True
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)) or \
                np.array_equal(np.isnan(got), np.isnan(want)) and \
                np.array_equal(got[~np.isnan(got)].view(np.uint32), want[~np.isnan(want)].view(np.uint32)), (src, regs)
        assert ok_once or src.count("(") > 20, src
    assert refused > 0  # some expressions need more than one or two registers


def test_expression_grammar_agrees_with_oracle(lib):
    """sg_fn_expr accepts exactly the texts the oracle's parser accepts."""
    from ctypes import byref, c_void_p
    from oracle.expr import parse
    L = lib.load()
    texts = ["x", "x+", "(x", "x)", "2x", "1e3*x", "1e*x", ".5*x", "5.*x", "x**2", "sin(x)", "sqrt x", "exp((x))",
             "--x", "x--x", "abs()", "", "   x   ", "x/0", "y", "3.0e-2+x", "x*-2", "(((x)))", "x..5"]
    for t in texts:
        try:
            parse(t)
            oracle_ok = True
        except ValueError:
            oracle_ok = False
        h = c_void_p()
        st = L.sg_fn_expr(t.encode(), byref(h))
        assert (st == 0) == oracle_ok, (t, st)
        if st == 0:
            L.sg_fn_release(h)
