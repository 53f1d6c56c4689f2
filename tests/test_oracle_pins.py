"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, special values, brute force with exact rational or 200-bit arithmetic on small
inputs, IEEE float32 arithmetic done natively by numpy, and algebraic invariants."""
import math
import struct
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import reduce as R
from oracle import matrix as M
from oracle.elem import apply_fn, eval_pred, exp_rn32, wrap_i32

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---- independent brute-force helpers ------------------------------------------------------

def f32_from_bits(b):
    return np.array([b], dtype=np.uint32).view(np.float32)[0]


def rn32_of_fraction(q: Fraction) -> np.float32:
    """Round an exact rational to the nearest binary32 (ties to even) by comparing distances
    to the neighbouring binary32 values; overflow per IEEE (>= FLT_MAX + half ulp -> inf)."""
    if q == 0:
        return np.float32(0.0)
    neg = q < 0
    a = -q if neg else q
    top = Fraction(2) ** 128 - Fraction(2) ** 103
    if a >= top:
        return np.float32(-np.inf if neg else np.inf)
    c = np.float32(float(a))
    cands = {c, np.nextafter(c, np.float32(0)), np.nextafter(c, np.float32(np.inf))}
    best = None
    for v in cands:
        if not np.isfinite(v):
            continue
        d = abs(Fraction(float(v)) - a)
        key = (d, int(np.float32(v).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, v)
    r = np.float32(best[1])
    return np.float32(-r) if neg else r


def mp_fraction(v) -> Fraction:
    m, e = v.man_exp
    return Fraction(int(m)) * (Fraction(2) ** int(e)) if e >= 0 else Fraction(int(m), 2 ** (-int(e)))


def exp_brute(t: np.float32) -> np.float32:
    t = float(t)
    if math.isnan(t):
        return np.float32(np.nan)
    if t == -math.inf:
        return np.float32(0.0)
    if t == math.inf:
        return np.float32(np.inf)
    mpmath.mp.prec = 240
    return rn32_of_fraction(mp_fraction(mpmath.exp(mpmath.mpf(t))))


def same_f32(a, b):
    a, b = np.float32(a), np.float32(b)
    if np.isnan(a) or np.isnan(b):
        return bool(np.isnan(a) and np.isnan(b))
    return a.view(np.uint32) == b.view(np.uint32)


# ---- exp ----------------------------------------------------------------------------------

def test_exp_special_values():
    t = np.array([0.0, -0.0, -np.inf, np.inf, np.nan, 1e-30, -1e-30], dtype=np.float32)
    out = exp_rn32(t)
    assert same_f32(out[0], 1.0) and same_f32(out[1], 1.0)
    assert same_f32(out[2], 0.0) and same_f32(out[3], np.inf) and np.isnan(out[4])
    assert same_f32(out[5], 1.0) and same_f32(out[6], 1.0)


def test_exp_overflow_and_underflow_edges():
    # around ln(FLT_MAX + ulp/2) ~ 88.7228 and around ln(2^-150) ~ -103.97
    lo = np.float32(88.7215)
    t = [lo]
    for _ in range(400):
        t.append(np.nextafter(t[-1], np.float32(np.inf)))
    t += [np.float32(-103.9), np.float32(-103.97), np.float32(-103.98), np.float32(-104.0),
          np.float32(-87.3365), np.float32(-87.33655)]
    t = np.array(t, dtype=np.float32)
    out = exp_rn32(t)
    for ti, oi in zip(t, out):
        assert same_f32(oi, exp_brute(ti)), (ti, oi)
    assert np.isinf(out[:401]).any() and np.isfinite(out[:401]).any()


def test_exp_random_sample_vs_240bit():
    g = np.random.default_rng(1234)
    t = np.concatenate([g.uniform(-104, 89, 1500), g.uniform(-1, 1, 500),
                        -(g.standard_normal(500) ** 2)]).astype(np.float32)
    out = exp_rn32(t)
    for ti, oi in zip(t, out):
        assert same_f32(oi, exp_brute(ti)), (ti, oi)


def test_exp_hard_cases_vs_240bit():
    """The elements whose float64 exp lies within 2^-40 of a binary32 rounding boundary are
    exactly where a float64-then-round shortcut could be wrong: check each by brute force."""
    t = W.uniform_f32(1 << 21, 777, -104.0, 89.0)
    out, hard = exp_rn32(t, return_hard=True)
    assert len(hard) > 5
    for i in hard:
        assert same_f32(out[i], exp_brute(t[i])), (t[i], out[i])


def test_exp_neg_sq_composition():
    u = W.normal_f32(300, 5, 3.0)
    out, dt = apply_fn(["exp_neg_sq"], u, "f32")
    assert dt == "f32"
    for ui, oi in zip(u, out):
        sq = np.float32(ui) * np.float32(ui)  # IEEE binary32 multiply
        assert same_f32(oi, exp_brute(-sq))


# ---- element-wise arithmetic --------------------------------------------------------------

def test_affine_matches_native_float32_ops():
    x = W.normal_f32(10000, 3, 10.0)
    a, b = np.float32(1.37), np.float32(-0.71)
    got, _ = apply_fn(["affine", float(a), float(b)], x, "f32")
    want = (a * x) + b  # numpy binary32 arithmetic, each op correctly rounded
    assert np.array_equal(got.view(np.uint32), want.astype(np.float32).view(np.uint32))


def test_affine_identity_and_dyadic_exact():
    x = W.uniform_f32(4096, 9)
    got, _ = apply_fn(["affine", 1.0, 0.0], x, "f32")
    assert np.array_equal(got, x)
    got, _ = apply_fn(["affine", 2.0, 1.0], x, "f32")
    for xi, gi in zip(x[:200], got[:200]):
        assert Fraction(float(gi)) == 2 * Fraction(float(xi)) + 1


def test_zip_add_neg_is_zero_and_native_ops():
    x = W.normal_f32(5000, 4)
    spec = {"inputs": [{"name": "x", "dtype": "f32", "n": 5000}, {"name": "y", "dtype": "f32", "n": 5000}],
            "nodes": [{"name": "z", "op": "zip", "a": "x", "b": "y", "binop": "add"},
                      {"name": "p", "op": "zip", "a": "x", "b": "y", "binop": "mul"},
                      {"name": "d", "op": "zip", "a": "x", "b": "y", "binop": "sub"}],
            "contracts": [], "outputs": ["z"]}
    r = oracle.evaluate(spec, {"x": x, "y": -x})
    assert np.all(r.values["z"] == 0)
    y = W.normal_f32(5000, 5)
    r = oracle.evaluate(spec, {"x": x, "y": y})
    assert np.array_equal(r.values["z"], x + y)
    assert np.array_equal(r.values["p"], x * y)
    assert np.array_equal(r.values["d"], x - y)


def test_sqrt_matches_native():
    x = W.normal_f32(20000, 6, 100.0)
    got, _ = apply_fn(["sqrt_abs"], x, "f32")
    assert np.array_equal(got, np.sqrt(np.abs(x)))


def test_i32_wraps_like_python_ints():
    x = W.uniform_i32(2000, 8)
    got, _ = apply_fn(["affine", 1103515245, 12345], x, "i32")
    for xi, gi in zip(x.tolist(), got.tolist()):
        v = (1103515245 * xi + 12345) % 2**32
        v = v - 2**32 if v >= 2**31 else v
        assert v == gi
    assert wrap_i32(np.array([2**31]))[0] == -(2**31)


def test_predicates_and_nan():
    x = np.array([np.nan, -np.inf, -1.0, -0.0, 0.0, 0.1, 1.0, np.inf], dtype=np.float32)
    assert eval_pred(["isfinite"], x, "f32").tolist() == [False, False, True, True, True, True, True, False]
    assert eval_pred(["cmp", "gt", 0.1], x, "f32").tolist() == [False] * 6 + [True, True]
    assert eval_pred(["cmp", "ge", 0.1], x, "f32").tolist() == [False] * 5 + [True] * 3
    assert eval_pred(["cmp", "ne", 0.0], x, "f32").tolist() == [True, True, True, False, False, True, True, True]
    assert eval_pred(["in_range", -1, 1], x, "f32").tolist() == [False, False, True, True, True, True, True, False]
    p = ["and", ["isfinite"], ["not", ["cmp", "lt", 0.0]]]
    assert eval_pred(p, x, "f32").tolist() == [False, False, False, True, True, True, True, False]
    # 0.1 is rounded to binary32 (0x3DCCCCCD) before comparing
    c = f32_from_bits(0x3DCCCCCD)
    y = np.array([c, np.nextafter(c, np.float32(1))], dtype=np.float32)
    assert eval_pred(["cmp", "gt", 0.1], y, "f32").tolist() == [False, True]


# ---- reductions ---------------------------------------------------------------------------

def test_sum_closed_forms():
    for n in (1, 2, 1000, 1 << 20, 1 << 24):
        x = np.arange(1, n + 1, dtype=np.float32)
        assert R.exact_sum_f32(x) == n * (n + 1) // 2
    assert R.exact_sum(np.arange(1, (1 << 20) + 1, dtype=np.float32), "f32") == 549756338176.0
    x = W.normal_f32(100001, 1, 1e3)
    inter = np.empty(2 * x.size, np.float32)
    inter[0::2], inter[1::2] = x, -x
    assert R.exact_sum_f32(inter) == 0
    c = np.full(1 << 16, 2.0 ** -140, dtype=np.float32)  # subnormal constants
    assert R.exact_sum_f32(c) == Fraction(1 << 16, 2 ** 140)


def test_sum_vs_fsum_and_fractions():
    for seed in range(5):
        x = W.normal_f32(50000, 100 + seed, 10.0 ** (seed - 2))
        assert R.exact_sum(x, "f32") == math.fsum(x.tolist())
    x = np.concatenate([W.normal_f32(50, 7), np.array([3e38, -3e38, 1e-45, -2e-44], np.float32)])
    assert R.exact_sum_f32(x) == sum(Fraction(float(v)) for v in x)


def test_int_sum_exact():
    x = W.uniform_i32(100000, 17)
    assert R.exact_sum(x, "i32") == sum(int(v) for v in x.tolist())


def test_max_min_total_order():
    x = np.array([-0.0, 0.0, -0.0], np.float32)
    assert same_f32(R.fmax_total(x), 0.0) and same_f32(R.fmin_total(x), -0.0)
    assert same_f32(R.fmax_total(np.array([-0.0, -1.0], np.float32)), -0.0)
    assert np.isnan(R.fmax_total(np.array([1.0, np.nan, 2.0], np.float32)))
    assert np.isnan(R.fmin_total(np.array([1.0, np.nan, 2.0], np.float32)))
    g = np.random.default_rng(3)
    for _ in range(50):
        x = g.standard_normal(g.integers(1, 60)).astype(np.float32)
        best = x[0]
        for v in x[1:]:
            best = v if v > best else best
        assert same_f32(R.fmax_total(x), best)


# ---- quantifiers and sortedness -----------------------------------------------------------

def test_quantifiers_brute_force_and_de_morgan():
    g = np.random.default_rng(11)
    for _ in range(200):
        n = int(g.integers(0, 40))
        p = g.random(n) < g.random()
        h, i = R.for_all(p)
        bad = [k for k in range(n) if not p[k]]
        assert (h, i) == ((True, -1) if not bad else (False, bad[0]))
        h2, i2 = R.exists(~p)
        assert h2 == (not h) and i2 == i
    assert R.for_all(np.zeros(0, bool)) == (True, -1)
    assert R.exists(np.zeros(0, bool)) == (False, -1)


def test_is_sorted_pins():
    x = np.arange(100, dtype=np.int32) * 3
    assert R.is_sorted(x) == (True, -1)
    assert R.is_sorted(x[::-1].copy()) == (False, 0)
    assert R.is_sorted(np.array([5, 5, 5], np.int32)) == (True, -1)
    assert R.is_sorted(np.zeros(0, np.int32)) == (True, -1)
    assert R.is_sorted(np.zeros(1, np.int32)) == (True, -1)
    g = np.random.default_rng(2)
    for _ in range(100):
        n = int(g.integers(2, 300))
        y = np.arange(n, dtype=np.int32)
        i, j = sorted(g.choice(n, 2, replace=False))
        y[i], y[j] = y[j], y[i]
        assert R.is_sorted(y) == (False, int(i))
    f = np.array([1.0, 2.0, np.nan, 3.0], np.float32)
    assert R.is_sorted(f) == (False, 1)


def test_sorted_keys_generator_swaps():
    keys, swaps = W.sorted_keys_with_swaps(10000, 23, 24, 0.001)
    assert len(swaps) == 10
    h, i = R.is_sorted(keys)
    # brute force scan
    first = next((k for k in range(len(keys) - 1) if not keys[k] <= keys[k + 1]), -1)
    assert (h, i) == (first < 0, first)


# ---- matrices -----------------------------------------------------------------------------

def test_matmul_identity_permutation_integer():
    A = W.normal_f32(64 * 48, 31).reshape(64, 48)
    assert np.array_equal(M.matmul64(A, np.eye(48, dtype=np.float32)), A.astype(np.float64))
    P, perm = W.permutation_matrix_f32(48, 34)
    assert np.array_equal(M.matmul64(A, P), A[:, perm].astype(np.float64))
    g = np.random.default_rng(5)
    Ai = g.integers(-8, 9, size=(32, 4096))
    Bi = g.integers(-8, 9, size=(4096, 16))
    C = M.matmul64(Ai.astype(np.float32), Bi.astype(np.float32))
    assert np.array_equal(C, (Ai @ Bi).astype(np.float64))


def test_matmul_tiny_vs_fractions():
    A = W.normal_f32(12, 1).reshape(3, 4)
    B = W.normal_f32(20, 2).reshape(4, 5)
    C = M.matmul64(A, B)
    for i in range(3):
        for j in range(5):
            exact = sum(Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(4))
            assert abs(Fraction(float(C[i, j])) - exact) <= abs(exact) * Fraction(1, 2 ** 50) + Fraction(1, 2 ** 200)


def test_product_check_pins():
    g = np.random.default_rng(8)
    n = 96
    A = g.integers(-8, 9, size=(n, n)).astype(np.float32)
    B = g.integers(-8, 9, size=(n, n)).astype(np.float32)
    Rv = g.integers(-8, 9, size=(4, n)).astype(np.float32)
    C = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    h, i, m = M.product_check(C, A, B, Rv)
    assert (h, i, m) == (True, -1, 0.0)
    C2 = C.copy()
    C2[17, 5] += 1000.0
    C2[40, 2] += 1000.0
    h, i, m = M.product_check(C2, A, B, Rv)
    assert not h and i == 17 and m > 1e-3
    C3 = C.copy()
    C3[3, 3] = np.nan
    assert M.product_check(C3, A, B, Rv)[:2] == (False, 3)
    assert abs(M.gamma(4096) - 4.885e-4) < 1e-6


# ---- whole specifications and the contract protocol ---------------------------------------

def test_dot_product_listing():
    x, y = W.normal_f32(3000, 40), W.normal_f32(3000, 41)
    spec = {"inputs": [{"name": "a", "dtype": "f32", "n": 3000}, {"name": "b", "dtype": "f32", "n": 3000}],
            "nodes": [{"name": "ab", "op": "zip", "a": "a", "b": "b", "binop": "mul"},
                      {"name": "dot", "op": "reduce", "src": "ab", "red": "sum"}],
            "contracts": [], "outputs": ["dot"]}
    r = oracle.evaluate(spec, {"a": x, "b": y})
    exact = sum(Fraction(float(np.float32(p))) for p in (x * y))
    assert r.values["dot"]["exact"] == float(exact)


def test_filter_brute_force():
    g = np.random.default_rng(9)
    for _ in range(30):
        n = int(g.integers(0, 200))
        x = g.standard_normal(n).astype(np.float32)
        t = float(np.float32(g.uniform(-1, 1)))
        spec = {"inputs": [{"name": "x", "dtype": "f32", "n": n}],
                "nodes": [{"name": "k", "op": "filter", "src": "x", "pred": ["cmp", "gt", t]},
                          {"name": "nk", "op": "filter", "src": "x", "pred": ["not", ["cmp", "gt", t]]},
                          {"name": "c", "op": "reduce", "src": "k", "red": "count"}],
                "contracts": [], "outputs": ["k"]}
        r = oracle.evaluate(spec, {"x": x})
        want = [v for v in x.tolist() if v > t]
        assert r.values["k"].tolist() == want
        assert r.values["c"]["value"] + len(r.values["nk"]) == n


def test_contract_protocol_cfg1():
    n = 4096
    spec = W.cfg1_spec(n)
    inp = W.cfg1_inputs(n)
    r = oracle.evaluate(spec, inp)
    assert r.status == "ok" and [v.holds for v in r.verdicts] == [1, 1, 1]
    x = inp["x"].copy()
    x[700] = np.nan
    x[900] = np.inf
    r = oracle.evaluate(spec, {"x": x, "y": inp["y"]})
    assert r.status == "pre_violated" and r.violated == 0
    assert r.verdicts[0].first_index == 700 and [v.holds for v in r.verdicts[1:]] == [-1, -1]
    assert r.values == {}
    y = inp["y"].copy()
    y[123] = 5.0
    y[3000] = -9.0
    r = oracle.evaluate(spec, {"x": inp["x"], "y": y})
    assert r.status == "post_violated" and r.violated == 1 and r.verdicts[1].first_index == 123
    r = oracle.evaluate(spec, {"x": x, "y": y}, mode="off")
    assert r.status == "ok" and all(v.holds == -1 for v in r.verdicts)
    r = oracle.evaluate(spec, {"x": inp["x"], "y": y}, mode="pre")
    assert r.status == "ok" and [v.holds for v in r.verdicts] == [1, -1, -1]


def test_closed_form_chain():
    """z = (2x+1) + y with x = 0..n-1 and y = -2x gives z = 1 everywhere, sum n."""
    n = 5000
    x = np.arange(n, dtype=np.float32)
    y = (-2 * x).astype(np.float32)
    spec = W.cfg1_spec(n)
    spec["contracts"] = []
    r = oracle.evaluate(spec, {"x": x, "y": y})
    assert r.values["s"]["exact"] == n and np.all(r.values["z"] == 1)


def test_i32_chain_and_sum():
    x = W.uniform_i32(1000, 3)
    spec = {"inputs": [{"name": "x", "dtype": "i32", "n": 1000}],
            "nodes": [{"name": "a", "op": "map", "src": "x", "fn": ["add_c", 7]},
                      {"name": "s", "op": "reduce", "src": "a", "red": "sum"},
                      {"name": "m", "op": "reduce", "src": "a", "red": "max"}],
            "contracts": [], "outputs": ["s"]}
    r = oracle.evaluate(spec, {"x": x})
    vals = [((v + 7 + 2**31) % 2**32) - 2**31 for v in x.tolist()]
    assert r.values["s"]["value"] == sum(vals) and r.values["m"]["value"] == max(vals)
