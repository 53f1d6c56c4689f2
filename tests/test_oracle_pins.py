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


# ---- every remaining element function, int32 op and predicate, and avg ------------------
#
# Each branch of apply_fn and eval_pred is compared with a definition computed a different
# way: exact rationals rounded by brute force (rn32_of_fraction), bit manipulation for the
# sign operations, C two's-complement truncation (ctypes) for int32 wrap-around, and Python
# comparisons in explicit loops for predicates.

import ctypes


def finite_f32_sample():
    """Normal, large, tiny and subnormal binary32 values, both signs, plus exact edge values."""
    g = np.random.Generator(np.random.PCG64(77))
    parts = [W.normal_f32(300, 1), W.normal_f32(100, 2, 1e18), W.normal_f32(100, 3, 1e-20),
             (g.integers(1, 1 << 23, 100).astype(np.uint32)).view(np.float32),            # +subnormals
             (g.integers(1, 1 << 23, 100).astype(np.uint32) | 0x80000000).view(np.float32),  # -subnormals
             np.array([0.0, -0.0, 1.0, -1.0, 0.5, 3.0, 1.17549435e-38, -1.17549435e-38, 3.4028235e38,
                       -3.4028235e38, 1.8446744e19, 2.0 ** -75, 2.0 ** -76], np.float32)]
    return np.concatenate(parts).astype(np.float32)


def bits(a):
    return np.asarray(a, np.float32).view(np.uint32)


def rn32_product(x, y):
    """IEEE product: the exact product rounded; a zero result (exact or underflowed) carries
    the exclusive-or of the operands' signs."""
    r = rn32_of_fraction(Fraction(float(x)) * Fraction(float(y)))
    if r == 0:
        return np.float32(-0.0) if np.signbit(x) != np.signbit(y) else np.float32(0.0)
    return r


def rn32_sum(x, y):
    """IEEE sum: the exact sum rounded; an exact zero is +0 unless both operands are -0."""
    q = Fraction(float(x)) + Fraction(float(y))
    if q == 0:
        return np.float32(-0.0) if (np.signbit(x) and np.signbit(y)) else np.float32(0.0)
    return rn32_of_fraction(q)


def test_f32_square_add_mul_c_vs_exact_rationals():
    x = finite_f32_sample()
    sq, _ = apply_fn(["square"], x, "f32")
    for xi, yi in zip(x, sq):
        assert same_f32(yi, rn32_product(xi, xi)), (xi, yi)
    for c in (0.1, -3.75, 1e-30, 7e25, -0.0):
        c32 = np.float32(c)
        ya, _ = apply_fn(["add_c", c], x, "f32")
        ym, _ = apply_fn(["mul_c", c], x, "f32")
        for xi, a, m in zip(x, ya, ym):
            assert same_f32(a, rn32_sum(xi, c32)), (xi, c, a)
            assert same_f32(m, rn32_product(xi, c32)), (xi, c, m)


def test_f32_neg_abs_are_sign_bit_operations():
    x = np.concatenate([finite_f32_sample(), np.array([np.inf, -np.inf, np.nan], np.float32)])
    neg, _ = apply_fn(["neg"], x, "f32")
    ab, _ = apply_fn(["abs"], x, "f32")
    assert np.array_equal(bits(neg), bits(x) ^ np.uint32(0x80000000))
    assert np.array_equal(bits(ab), bits(x) & np.uint32(0x7FFFFFFF))


def test_f32_sqrt_brackets_the_exact_root():
    """r = RN32(sqrt(x)) iff x lies strictly between the squares of the midpoints around r
    (no ties are possible for sqrt of a binary32 value)."""
    x = np.abs(finite_f32_sample())
    r, _ = apply_fn(["sqrt"], x, "f32")
    for xi, ri in zip(x, r):
        X = Fraction(float(xi))
        if X == 0:
            assert ri == 0 and np.signbit(ri) == np.signbit(xi)
            continue
        lo = (Fraction(float(ri)) + Fraction(float(np.nextafter(ri, np.float32(0))))) / 2
        hi = (Fraction(float(ri)) + Fraction(float(np.nextafter(ri, np.float32(np.inf))))) / 2
        assert lo * lo < X < hi * hi, (xi, ri)
    sp, _ = apply_fn(["sqrt"], np.array([-1.0, -1e-40, np.inf, np.nan, -0.0], np.float32), "f32")
    assert np.isnan(sp[0]) and np.isnan(sp[1]) and sp[2] == np.inf and np.isnan(sp[3])
    assert sp[4] == 0 and np.signbit(sp[4])
    sa, _ = apply_fn(["sqrt_abs"], np.array([-4.0, -0.0, -np.inf], np.float32), "f32")
    assert sa.tolist() == [2.0, 0.0, np.inf] and not np.signbit(sa[1])


def test_f32_special_values_follow_ieee():
    x = np.array([np.inf, -np.inf, np.nan], np.float32)
    sq, _ = apply_fn(["square"], x, "f32")
    assert sq[0] == np.inf and sq[1] == np.inf and np.isnan(sq[2])
    m0, _ = apply_fn(["mul_c", 0.0], x, "f32")
    assert np.all(np.isnan(m0))                     # inf * 0 is invalid
    a, _ = apply_fn(["add_c", -1e30], x, "f32")
    assert a[0] == np.inf and a[1] == -np.inf and np.isnan(a[2])
    big, _ = apply_fn(["square"], np.array([1e20, -2e19], np.float32), "f32")
    assert np.all(big == np.inf)                     # overflow rounds to infinity


def test_i2f_rounds_exact_integers_to_nearest_even():
    g = np.random.Generator(np.random.PCG64(78))
    v = np.concatenate([g.integers(-2**31, 2**31, 3000).astype(np.int64),
                        np.array([0, 1, -1, 2**24, 2**24 + 1, 2**24 + 3, -(2**24 + 1), 2**31 - 1, -2**31,
                                  16777217, 33554435, 2**30 + 64, 2**30 + 65])]).astype(np.int32)
    got, dt = apply_fn(["i2f"], v, "i32")
    assert dt == "f32"
    for vi, gi in zip(v.tolist(), got):
        assert same_f32(gi, rn32_of_fraction(Fraction(vi))), (vi, gi)
    # the halfway case 2^24 + 1 rounds to the even neighbour 2^24
    assert float(apply_fn(["i2f"], np.array([2**24 + 1], np.int32), "i32")[0][0]) == 2.0 ** 24


def c_i32(v: int) -> int:
    return ctypes.c_int32(v).value  # C conversion to a 32-bit two's-complement integer


def test_i32_square_neg_abs_add_mul_wrap_like_c():
    g = np.random.Generator(np.random.PCG64(79))
    x = np.concatenate([g.integers(-2**31, 2**31, 2000),
                        np.array([0, 1, -1, 46340, 46341, -46341, 65536, 2**31 - 1, -2**31])]).astype(np.int32)
    cases = {"square": lambda a: a * a, "neg": lambda a: -a, "abs": lambda a: abs(a),
             ("add_c", 2**31 - 5): lambda a: a + (2**31 - 5), ("mul_c", -7919): lambda a: a * -7919,
             ("affine", 65537, -3): lambda a: 65537 * a - 3}
    for key, f in cases.items():
        fn = [key] if isinstance(key, str) else list(key)
        got, dt = apply_fn(fn, x, "i32")
        assert dt == "i32"
        assert [c_i32(f(int(a))) for a in x.tolist()] == got.tolist(), fn
    # the edge cases a two's-complement machine produces
    assert apply_fn(["neg"], np.array([-2**31], np.int32), "i32")[0][0] == -2**31
    assert apply_fn(["abs"], np.array([-2**31], np.int32), "i32")[0][0] == -2**31


def test_i32_predicate_truth_table():
    vals = [-2**31, -1000, -5, -1, 0, 1, 5, 1000, 2**31 - 1]
    x = np.array(vals, np.int32)
    py = {"lt": lambda a, c: a < c, "le": lambda a, c: a <= c, "gt": lambda a, c: a > c,
          "ge": lambda a, c: a >= c, "eq": lambda a, c: a == c, "ne": lambda a, c: a != c}
    for op, f in py.items():
        for c in (-5, 0, 1, 2**31 - 1, -2**31):
            assert eval_pred(["cmp", op, c], x, "i32").tolist() == [f(a, c) for a in vals], (op, c)
    assert eval_pred(["in_range", -5, 5], x, "i32").tolist() == [-5 <= a <= 5 for a in vals]
    assert eval_pred(["isfinite"], x, "i32").tolist() == [True] * len(vals)
    assert eval_pred(["true"], x, "i32").tolist() == [True] * len(vals)
    p = ["or", ["cmp", "lt", -999], ["and", ["cmp", "ge", 0], ["not", ["cmp", "eq", 5]]]]
    assert eval_pred(p, x, "i32").tolist() == [(a < -999) or (a >= 0 and not a == 5) for a in vals]
    with pytest.raises(ValueError):
        eval_pred(["cmp", "gt", 0.5], x, "i32")  # an int predicate constant must be integral


def avg_spec(n, dtype, filt=None):
    nodes = []
    src = "x"
    if filt is not None:
        nodes.append({"name": "k", "op": "filter", "src": "x", "pred": filt})
        src = "k"
    nodes.append({"name": "a", "op": "reduce", "src": src, "red": "avg"})
    return {"inputs": [{"name": "x", "dtype": dtype, "n": n}], "nodes": nodes, "contracts": [], "outputs": ["a"]}


def test_avg_closed_forms_and_empty():
    for n in (1, 2, 999, 1000, 1 << 20):
        x = np.arange(1, n + 1, dtype=np.float32)
        r = oracle.evaluate(avg_spec(n, "f32"), {"x": x}).values["a"]
        assert r["exact"] == (n + 1) / 2 and r["value"] == (n + 1) / 2  # exact in binary32
        xi = np.arange(1, n + 1, dtype=np.int32)
        ri = oracle.evaluate(avg_spec(n, "i32"), {"x": xi}).values["a"]
        assert Fraction(ri["exact"]) == Fraction(n + 1, 2)
    for dt, arr in (("f32", np.zeros(0, np.float32)), ("i32", np.zeros(0, np.int32))):
        r = oracle.evaluate(avg_spec(0, dt), {"x": arr}).values["a"]
        assert math.isnan(r["value"]) and math.isnan(r["exact"])
    # everything filtered out: the mean of an empty collection
    x = W.uniform_f32(1000, 5)
    r = oracle.evaluate(avg_spec(1000, "f32", ["cmp", "gt", 2.0]), {"x": x}).values["a"]
    assert math.isnan(r["value"])


def test_avg_filtered_vs_fraction_mean():
    x = W.normal_f32(5001, 6)
    r = oracle.evaluate(avg_spec(5001, "f32", ["cmp", "gt", 0.25]), {"x": x}).values["a"]
    kept = [Fraction(float(v)) for v in x if float(v) > float(np.float32(0.25))]
    mean = sum(kept, Fraction(0)) / len(kept)
    assert r["exact"] == float(mean)                      # correctly rounded float64 mean
    assert abs(Fraction(r["value"]) - mean) <= Fraction(float(abs(np.float32(r["value"])))) / 2**23
    assert r["abs_sum"] == float(sum((abs(k) for k in kept), Fraction(0)))
    xi = W.uniform_i32(4003, 7, -10**6, 10**6)
    ri = oracle.evaluate(avg_spec(4003, "i32", ["cmp", "lt", 0]), {"x": xi}).values["a"]
    neg = [int(v) for v in xi.tolist() if v < 0]
    assert ri["exact"] == float(Fraction(sum(neg), len(neg)))
