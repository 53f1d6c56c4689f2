"""Element functions and predicates of the oracle (agents applied per element).

Follows the collection API's project/filter/for_all/exists (Section 3.2, Table 2) and the
vector operations of Section 3.3.  The paper leaves precision and rounding open; the
reading taken here is: every float32 node value is the round-to-nearest-even binary32 of
the exact result of its operation on already-rounded binary32 operands; int32 arithmetic
wraps modulo 2^32; constants are rounded to the node's element type when the chain is
composed.

For + - x and sqrt, evaluating in float64 and rounding once to float32 gives the correctly
rounded float32 result (double rounding is innocuous because 53 >= 2*24 + 2).  exp has no
such guarantee, so ``exp_rn32`` resolves the cases where float64 lands too close to a
float32 rounding boundary with 200-bit mpmath arithmetic.
"""
from __future__ import annotations

import numpy as np

try:
    import mpmath
except ImportError:  # pragma: no cover - mpmath ships with the image
    mpmath = None

F32_MAX = float(np.finfo(np.float32).max)
TWO128 = 2.0 ** 128
# float64 exp in numpy has a relative error far below this; within this distance of a
# binary32 rounding boundary the result is recomputed with mpmath.
HARD_BAND = 2.0 ** -40


def wrap_i32(v: np.ndarray) -> np.ndarray:
    """int64 -> int32 modulo 2^32 (two's complement wrap)."""
    v = np.asarray(v, dtype=np.int64)
    return (((v + 2**31) % 2**32) - 2**31).astype(np.int32)


def _rn32(v64: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore", invalid="ignore"):
        return np.asarray(v64, dtype=np.float64).astype(np.float32)


def _bracket(y: np.ndarray):
    """For float64 y >= 0 return float64 (a, b): consecutive binary32 values with a <= y <= b,
    where the value after FLT_MAX is taken as 2^128 (the overflow boundary)."""
    f = _rn32(y)
    f64 = f.astype(np.float64)
    up = np.nextafter(f, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(f, np.float32(-np.inf)).astype(np.float64)
    up = np.where(np.isinf(up) & np.isfinite(f64), TWO128, up)
    below = f64 <= y
    a = np.where(below, f64, dn)
    b = np.where(below, up, f64)
    # f == +inf: y lies in [FLT_MAX, inf)
    is_inf = np.isinf(f64)
    a = np.where(is_inf, F32_MAX, a)
    b = np.where(is_inf, TWO128, b)
    return a, b


def _exp_rn32_mp(t: float) -> np.float32:
    """Correctly rounded binary32 exp(t) for one finite binary32 t, by 200-bit arithmetic."""
    mpmath.mp.prec = 200
    v = mpmath.exp(mpmath.mpf(t))
    y = float(v)  # correctly rounded float64 of v
    a, b = _bracket(np.array([y]))
    a, b = float(a[0]), float(b[0])
    mid = mpmath.mpf(a) + (mpmath.mpf(b) - mpmath.mpf(a)) / 2
    if v < mpmath.mpf(a):
        return np.float32(a)
    if v > mpmath.mpf(b):
        return np.float32(b) if b != TWO128 else np.float32(np.inf)
    if v > mid:
        pick = b
    elif v < mid:
        pick = a
    else:  # exact tie: round to even significand (exp of a nonzero rational is never a tie)
        pick = a if (np.float32(a).view(np.uint32) & 1) == 0 else b
    return np.float32(np.inf) if pick == TWO128 else np.float32(pick)


def exp_rn32(t: np.ndarray, return_hard: bool = False):
    """Correctly rounded binary32 exp of a binary32 array."""
    t = np.asarray(t, dtype=np.float32)
    with np.errstate(over="ignore", under="ignore", invalid="ignore"):
        y = np.exp(t.astype(np.float64))
    out = _rn32(y)
    fin = np.isfinite(y) & (y > 0)
    a, b = _bracket(np.where(fin, y, 1.0))
    mid = a + (b - a) * 0.5  # exact: a and b are adjacent binary32 values (or FLT_MAX, 2^128)
    hard = fin & (np.abs(y - mid) <= HARD_BAND * y)
    # near the overflow boundary float64 exp itself is finite; also near zero (y tiny) the
    # bracket is exact, so the same test applies.
    idx = np.nonzero(hard)[0]
    for i in idx:
        out[i] = _exp_rn32_mp(float(t[i]))
    if return_hard:
        return out, idx
    return out


def _f64(x: np.ndarray) -> np.ndarray:
    return np.asarray(x).astype(np.float64)


def apply_fn(fn, x: np.ndarray, dtype: str):
    """Apply an element function (spec form) to the values of a node of element type dtype.
    Returns (values, out_dtype)."""
    name = fn[0]
    if name == "compose":
        v, d = apply_fn(fn[1], x, dtype)
        return apply_fn(fn[2], v, d)
    if name == "expr":
        if dtype != "f32":
            raise ValueError("expression functions are defined on f32")
        from .expr import apply_expr
        return apply_expr(fn[1], x), "f32"
    if dtype == "f32":
        xf = _f64(x)
        with np.errstate(all="ignore"):
            if name == "affine":
                a, b = np.float64(np.float32(fn[1])), np.float64(np.float32(fn[2]))
                t = _rn32(a * xf).astype(np.float64)
                return _rn32(t + b), "f32"
            if name == "add_c":
                return _rn32(xf + np.float64(np.float32(fn[1]))), "f32"
            if name == "mul_c":
                return _rn32(xf * np.float64(np.float32(fn[1]))), "f32"
            if name == "square":
                return _rn32(xf * xf), "f32"
            if name == "neg":
                return (-np.asarray(x, np.float32)).astype(np.float32), "f32"
            if name == "abs":
                return np.abs(np.asarray(x, np.float32)), "f32"
            if name == "sqrt":
                return _rn32(np.sqrt(xf)), "f32"
            if name == "sqrt_abs":
                return _rn32(np.sqrt(np.abs(xf))), "f32"
            if name == "exp":
                return exp_rn32(np.asarray(x, np.float32)), "f32"
            if name == "exp_neg_sq":
                sq = _rn32(xf * xf)
                return exp_rn32(-sq), "f32"
        raise ValueError(f"function {name} not defined on f32")
    if dtype == "i32":
        xi = np.asarray(x).astype(np.int64)
        if name == "affine":
            return wrap_i32(int(fn[1]) * xi + int(fn[2])), "i32"
        if name == "add_c":
            return wrap_i32(xi + int(fn[1])), "i32"
        if name == "mul_c":
            return wrap_i32(xi * int(fn[1])), "i32"
        if name == "square":
            return wrap_i32(xi * xi), "i32"
        if name == "neg":
            return wrap_i32(-xi), "i32"
        if name == "abs":
            return wrap_i32(np.abs(xi)), "i32"
        if name == "i2f":
            return _rn32(xi.astype(np.float64)), "f32"
        raise ValueError(f"function {name} not defined on i32")
    raise ValueError(dtype)


def _const(c, dtype):
    if dtype == "f32":
        return np.float64(np.float32(c))
    ci = int(c)
    if ci != c:
        raise ValueError("integer predicate constant must be integral")
    return ci


def eval_pred(pred, x: np.ndarray, dtype: str) -> np.ndarray:
    """Evaluate a predicate agent on every element; comparisons with NaN are false."""
    name = pred[0]
    v = _f64(x) if dtype == "f32" else np.asarray(x).astype(np.int64)
    with np.errstate(invalid="ignore"):
        if name == "true":
            return np.ones(len(v), dtype=bool)
        if name == "cmp":
            op, c = pred[1], _const(pred[2], dtype)
            # IEEE comparisons: every ordered comparison and eq is false for NaN, ne is true.
            return {"lt": v < c, "le": v <= c, "gt": v > c, "ge": v >= c,
                    "eq": v == c, "ne": v != c}[op]
        if name == "isfinite":
            return np.isfinite(v) if dtype == "f32" else np.ones(len(v), dtype=bool)
        if name == "in_range":
            lo, hi = _const(pred[1], dtype), _const(pred[2], dtype)
            return (v >= lo) & (v <= hi)
        if name == "and":
            return eval_pred(pred[1], x, dtype) & eval_pred(pred[2], x, dtype)
        if name == "or":
            return eval_pred(pred[1], x, dtype) | eval_pred(pred[2], x, dtype)
        if name == "not":
            return ~eval_pred(pred[1], x, dtype)
    raise ValueError(f"unknown predicate {name}")
