"""Matrix and vector operations of Sections 2.1, 3.3 and 3.4 in plain numpy: transposition,
matrix-vector products (right_multiply: M v; left_multiply: v M) and component-wise division
with its built-in contracts (Listing 2).

Readings:
* A matrix-vector product is the exact sum of exact float32 products, accumulated in float64
  (every float32 x float32 product is exact in float64); its float32 value is that sum rounded.
  Like the float sums, the device's value is accepted within 1e-5 of sum_k |M_ik v_k|.
* right_multiply(v) of an r x c matrix needs count(v) = c and gives an r x 1 matrix;
  left_multiply(v) needs count(v) = r and gives a 1 x c matrix (Listing 1's require and ensure:
  dimensions are scalar contracts, checked when the operation is composed).
* compwise_divide (Listing 2): require other.count = count (at composition) and
  other.for_all(item /= 0); ensure Result * other = Current.  The equality is read as IEEE
  float32 arithmetic allows: with q = RN(a / b) and p = RN(q * b), |p - a| <= 4u |a| +
  2^-149 |b| (u = 2^-24; the second term covers a quotient in the subnormal range), or p = a
  exactly (infinities).  'ensure Current = old Current' always holds: no operation changes its
  operands.
"""
from __future__ import annotations

import numpy as np

QUOT_REL = 2.0 ** -22     # 4u
QUOT_ABS = 2.0 ** -149    # times |b|


def transpose(M: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(M).T)


def matvec(M: np.ndarray, v: np.ndarray, side: str):
    """(float32 result, float64 exact-product sums, sum of |products|) of M v (side 'right')
    or v M (side 'left')."""
    M64 = np.asarray(M, np.float64)
    v64 = np.asarray(v, np.float64).reshape(-1)
    if side == "right":
        s, a = M64 @ v64, np.abs(M64) @ np.abs(v64)
    elif side == "left":
        s, a = v64 @ M64, np.abs(v64) @ np.abs(M64)
    else:
        raise ValueError(side)
    with np.errstate(over="ignore"):
        return s.astype(np.float32), s, a


def quotient_holds(q: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per element: does RN(q * b) reproduce a within the division's rounding bound?"""
    q, a, b = (np.asarray(x, np.float32) for x in (q, a, b))
    with np.errstate(all="ignore"):
        p = (q * b).astype(np.float32)  # one binary32 product
        d = np.abs(p.astype(np.float64) - a.astype(np.float64))
        bound = QUOT_REL * np.abs(a.astype(np.float64)) + QUOT_ABS * np.abs(b.astype(np.float64))
        return (p == a) | (d <= bound)
