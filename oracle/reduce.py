"""Reductions and range queries of the oracle.

Section 3.3 lists sum, avg, min, max and is_sorted on vectors; Section 3.2 (Table 2) defines
for_all and exists; Section 4 classifies them as range contracts.  The paper returns only a
Boolean from the quantifiers; this library also reports the first violating (for_all,
is_sorted) or witnessing (exists) index, 0-based, -1 when there is none.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_sum_f32(x: np.ndarray) -> Fraction | float:
    """Exact sum of finite binary32 values as a Fraction.

    Every binary32 value is m * 2^(e-150) with an integer |m| < 2^24 and 1 <= e <= 254, so
    the values are grouped by e, their integer significands summed exactly per group, and
    the groups combined with Python integers.  The significands are split into 12-bit
    halves so that the per-group float64 sums stay integers below 2^53 (exact) for up to
    2^41 elements.  Non-finite inputs return the IEEE result as a float.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.size == 0:
        return Fraction(0)
    if not np.all(np.isfinite(x)):
        with np.errstate(invalid="ignore", over="ignore"):
            return float(np.sum(x.astype(np.float64)))
    bits = x.view(np.uint32).astype(np.int64)
    neg = (bits >> 31) == 1
    E = (bits >> 23) & 0xFF
    m = bits & 0x7FFFFF
    m = np.where(E > 0, m | 0x800000, m)
    e = np.where(E > 0, E, 1)
    hi = (m >> 12).astype(np.float64)
    lo = (m & 0xFFF).astype(np.float64)
    sgn = np.where(neg, -1.0, 1.0)
    s_hi = np.bincount(e, weights=sgn * hi, minlength=256)
    s_lo = np.bincount(e, weights=sgn * lo, minlength=256)
    total = 0
    for k in range(256):
        if s_hi[k] != 0.0 or s_lo[k] != 0.0:
            total += ((int(s_hi[k]) << 12) + int(s_lo[k])) << k
    return Fraction(total, 1 << 150)


def exact_sum(x: np.ndarray, dtype: str):
    """Sum of a collection: the exact sum (as float64, correctly rounded) for f32, the exact
    int64 sum for i32."""
    if dtype == "i32":
        return int(np.sum(np.asarray(x).astype(np.int64)))
    s = exact_sum_f32(x)
    return float(s) if isinstance(s, Fraction) else s


def abs_sum(x: np.ndarray, dtype: str):
    if dtype == "i32":
        return int(np.sum(np.abs(np.asarray(x).astype(np.int64))))
    return exact_sum(np.abs(np.asarray(x, np.float32)), "f32")


def fmax_total(x: np.ndarray) -> np.float32:
    """Maximum of float32 values: NaN if any element is NaN, and -0 < +0."""
    x = np.asarray(x, np.float32)
    if np.any(np.isnan(x)):
        return np.float32(np.nan)
    m = np.max(x)
    if m == 0:
        return np.float32(0.0) if np.any((x == 0) & ~np.signbit(x)) else np.float32(-0.0)
    return np.float32(m)


def fmin_total(x: np.ndarray) -> np.float32:
    """Minimum of float32 values: NaN if any element is NaN, and -0 < +0."""
    x = np.asarray(x, np.float32)
    if np.any(np.isnan(x)):
        return np.float32(np.nan)
    m = np.min(x)
    if m == 0:
        return np.float32(-0.0) if np.any((x == 0) & np.signbit(x)) else np.float32(0.0)
    return np.float32(m)


def for_all(p: np.ndarray) -> tuple[bool, int]:
    """(holds, first index where the predicate is false or -1); empty -> (True, -1)."""
    p = np.asarray(p, dtype=bool)
    bad = np.nonzero(~p)[0]
    return (True, -1) if bad.size == 0 else (False, int(bad[0]))


def exists(p: np.ndarray) -> tuple[bool, int]:
    """(holds, first index where the predicate is true or -1); empty -> (False, -1)."""
    p = np.asarray(p, dtype=bool)
    good = np.nonzero(p)[0]
    return (False, -1) if good.size == 0 else (True, int(good[0]))


def is_sorted(x: np.ndarray) -> tuple[bool, int]:
    """Non-decreasing order: holds iff x[i] <= x[i+1] for all i; the reported index is the
    left element of the first pair that fails (a NaN makes its pairs fail)."""
    x = np.asarray(x)
    if x.size <= 1:
        return True, -1
    with np.errstate(invalid="ignore"):
        ok = x[:-1] <= x[1:]
    return for_all(ok)
