"""Pins of the expression agents: the same formulas written out in numpy's native binary32
arithmetic (each operation correctly rounded by IEEE 754), exact rationals rounded step by
step, the correctly rounded exp on brute-force points, grammar precedence, literal rounding
and rejected inputs."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle.expr import apply_expr, parse
from test_oracle_pins import exp_brute, rn32_of_fraction, same_f32

F = np.float32


def native_cases(x):
    """(expression, value computed with numpy float32 operations written by hand)"""
    with np.errstate(all="ignore"):
        return [
            ("x*0.3+0.7", x * F(0.3) + F(0.7)),
            ("0.7+x*0.3", F(0.7) + x * F(0.3)),
            ("(x-1.5)/(x+2)", (x - F(1.5)) / (x + F(2))),
            ("x*x - 3*x + 2", (x * x - F(3) * x) + F(2)),
            ("-x/7", (-x) / F(7)),
            ("2-x-x*x", (F(2) - x) - x * x),
            ("1/(1+x*x)", F(1) / (F(1) + x * x)),
            ("sqrt(abs(x))*0.5", np.sqrt(np.abs(x)) * F(0.5)),
            ("abs(x-0.25)", np.abs(x - F(0.25))),
            ("1e-3*x/3.0e2", (F(1e-3) * x) / F(300)),
        ]


def test_matches_native_float32_arithmetic():
    x = np.concatenate([W.normal_f32(3000, 1, 3.0), np.array([0, -0.0, 1, -1, 2, np.inf, -np.inf, np.nan], F)])
    for src, want in native_cases(x):
        got = apply_expr(src, x)
        assert got.dtype == np.float32
        nan = np.isnan(want)
        assert np.array_equal(np.isnan(got), nan), src
        assert np.array_equal(got[~nan].view(np.uint32), want.astype(F)[~nan].view(np.uint32)), src


def test_step_by_step_exact_rationals():
    x = W.normal_f32(200, 2, 10.0)
    got = apply_expr("(x*1.25 - 0.1) / (x + 3.3)", x)
    c1, c2, c3 = (Fraction(float(F(v))) for v in (1.25, 0.1, 3.3))
    for xi, gi in zip(x, got):
        X = Fraction(float(xi))
        a = rn32_of_fraction(X * c1)
        b = rn32_of_fraction(Fraction(float(a)) - c2)
        d = rn32_of_fraction(X + c3)
        assert same_f32(gi, rn32_of_fraction(Fraction(float(b)) / Fraction(float(d))))


def test_exp_is_correctly_rounded():
    t = np.array([-3.7, 0.0, 1.5, -88.0, 10.25, -0.001], F)
    got = apply_expr("exp(x*2-1)", t)
    for ti, gi in zip(t, got):
        arg = rn32_of_fraction(Fraction(float(rn32_of_fraction(Fraction(float(ti)) * 2))) - 1)
        assert same_f32(gi, exp_brute(arg))


def test_grammar():
    x = np.array([5.0], F)
    assert apply_expr("8/2/2", x)[0] == 2.0       # left associative
    assert apply_expr("2-3-4", x)[0] == -5.0
    assert apply_expr("2+3*4", x)[0] == 14.0      # * before +
    assert apply_expr("(2+3)*4", x)[0] == 20.0
    assert apply_expr("2*-x", x)[0] == -10.0      # unary minus
    assert apply_expr("--x", x)[0] == 5.0
    assert parse("0.1") == ("const", float(F(0.1)))  # literals rounded to binary32
    assert apply_expr(" x ", x)[0] == 5.0
    for bad in ("x+", "foo(x)", "x**2", "(x", "x)", "", "y", "1 2", "sqrt x"):
        with pytest.raises(ValueError):
            parse(bad)
