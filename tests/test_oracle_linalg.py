"""Pins of the matrix/vector oracle: transposition by index brute force, matrix-vector products
against identity, integer and exact-rational cases, component-wise division against exact
rationals, and Listing 2's built-in contracts on hand-made cases."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.linalg import matvec, quotient_holds, transpose
from test_oracle_pins import rn32_of_fraction, same_f32


def test_transpose_brute_force():
    M = W.normal_f32(7 * 13, 1).reshape(7, 13)
    T = transpose(M)
    assert T.shape == (13, 7)
    for i in range(7):
        for j in range(13):
            assert T[j, i] == M[i, j]
    assert np.array_equal(transpose(T), M)


def test_matvec_identity_integer_and_exact():
    v = W.normal_f32(64, 2)
    I = np.eye(64, dtype=np.float32)
    for side in ("right", "left"):
        r, _, _ = matvec(I, v, side)
        assert np.array_equal(r.reshape(-1), v)
    g = np.random.Generator(np.random.PCG64(3))
    M = g.integers(-9, 10, (30, 40)).astype(np.float32)
    x = g.integers(-9, 10, 40).astype(np.float32)
    r, s, a = matvec(M, x, "right")
    assert np.array_equal(r, (M.astype(np.int64) @ x.astype(np.int64)).astype(np.float32))
    y = g.integers(-9, 10, 30).astype(np.float32)
    r, s, a = matvec(M, y, "left")
    assert np.array_equal(r, (y.astype(np.int64) @ M.astype(np.int64)).astype(np.float32))
    M = W.normal_f32(3 * 4, 4).reshape(3, 4)
    x = W.normal_f32(4, 5)
    _, s, a = matvec(M, x, "right")
    for i in range(3):
        ex = sum(Fraction(float(M[i, k])) * Fraction(float(x[k])) for k in range(4))
        assert abs(Fraction(s[i]) - ex) <= abs(ex) * Fraction(1, 2**50)
        assert a[i] == float(sum(abs(Fraction(float(M[i, k])) * Fraction(float(x[k]))) for k in range(4)))


def test_divide_matches_exact_rationals():
    a = W.normal_f32(400, 6, 1e3)
    b = W.normal_f32(400, 7, 1e-3)
    spec = {"inputs": [{"name": "a", "dtype": "f32", "n": 400}, {"name": "b", "dtype": "f32", "n": 400}],
            "nodes": [{"name": "q", "op": "zip", "a": "a", "b": "b", "binop": "div"}], "contracts": [],
            "outputs": ["q"]}
    r = oracle.evaluate(spec, {"a": a, "b": b})
    for ai, bi, qi in zip(a, b, r.values["q"]):
        assert same_f32(qi, rn32_of_fraction(Fraction(float(ai)) / Fraction(float(bi))))
    # Listing 2's clauses are there, ahead of the user's, and hold
    assert [v.holds for v in r.verdicts] == [1, 1]


def test_quotient_postcondition_hand_cases():
    a = np.array([1.0, 3.0, 1e-30, np.inf, 0.0, 2.0], np.float32)
    b = np.array([3.0, 3.0, 1e20, 2.0, 5.0, 1e-30], np.float32)
    q = (a / b).astype(np.float32)
    assert quotient_holds(q, a, b).all()
    bad = q.copy()
    for _ in range(8):  # 8 units in the last place of 1/3: 6u relative, beyond the 4u bound
        bad[0] = np.nextafter(bad[0], np.float32(1))
    ok = q.copy()
    ok[0] = np.nextafter(np.nextafter(q[0], np.float32(1)), np.float32(1))  # 1.5u: within
    assert quotient_holds(ok, a, b).all()
    bad[1] = np.float32(1.0001)
    assert quotient_holds(bad, a, b).tolist() == [False, False, True, True, True, True]
    assert not quotient_holds(np.array([np.nan], np.float32), np.array([1.0], np.float32),
                              np.array([2.0], np.float32))[0]


def test_builtin_clauses_order_and_zero_divisor():
    n = 100
    a, b, c = W.uniform_f32(n, 1), W.uniform_f32(n, 2), W.uniform_f32(n, 3)
    spec = {"inputs": [{"name": k, "dtype": "f32", "n": n} for k in "abc"],
            "nodes": [{"name": "q", "op": "zip", "a": "a", "b": "b", "binop": "div"},
                      {"name": "r", "op": "zip", "a": "q", "b": "c", "binop": "div"},
                      {"name": "s", "op": "reduce", "src": "r", "red": "sum"}],
            "contracts": [{"kind": "ensure", "check": "for_all", "node": "r", "pred": ["isfinite"]}],
            "outputs": ["s"]}
    bz = b.copy()
    bz[17] = 0.0
    bz[60] = -0.0
    r = oracle.evaluate(spec, {"a": a, "b": bz, "c": c})
    assert r.status == "pre_violated" and r.violated == 0
    assert (r.verdicts[0].holds, r.verdicts[0].first_index) == (0, 17)
    assert len(r.verdicts) == 5  # two built-in clauses per division, then the user's
    r = oracle.evaluate(spec, {"a": a, "b": b, "c": c})
    assert [v.holds for v in r.verdicts] == [1, 1, 1, 1, 1]
