"""Determinant by Gaussian elimination (Section 5, Listing 5), in plain numpy float64.

The listing eliminates column by column: the pivot row is scaled, and every later row has the
pivot row subtracted so that its entry below the pivot becomes zero; the determinant is the
product of the pivots.  As printed it does not compute a determinant (a row scaled by 1/q
changes the determinant by 1/q, and the listing never multiplies it back in; after a zero pivot
its loop bounds never meet), so the oracle takes the textbook form of the same elimination,
with partial pivoting so that a zero on the diagonal does not stop it early:

  for k = 0 .. n-1:
      p = the first row i >= k with the largest |W[i, k]| (a NaN counts as largest)
      if W[p, k] == 0: the matrix is singular, det = 0, stop
      swap rows p and k (each swap flips the sign)
      det *= W[k, k]
      for every row i > k:  l = W[i, k] / W[k, k];  W[i, j] = W[i, j] - l * W[k, j]  (j > k)

Every operation is one IEEE float64 operation on float64 values (float32 input widened exactly),
the product and the difference rounded separately (no fused multiply-add).  The product of the
pivots is kept as a mantissa in [0.5, 1) and a binary exponent, renormalized after every step
(exact: it only moves powers of two), so a determinant outside the float64 range is still
represented; det = sign * mantissa * 2^exponent.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_det(A: np.ndarray):
    """Returns (sign, mantissa, exponent, W): det = sign * mantissa * 2**exponent with the
    mantissa in [0.5, 1) (0.0 and exponent 0 for a singular matrix), and W the eliminated
    working matrix (float64; its upper triangle holds the pivots' rows)."""
    W = np.array(A, dtype=np.float64)
    if W.ndim != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("the determinant needs a square matrix (rows = columns)")
    n = W.shape[0]
    sign, mant, expo = 1, 0.5, 1  # the empty product 1 = 0.5 * 2^1
    for k in range(n):
        col = np.abs(W[k:, k])
        p = k + int(np.argmax(col))  # first maximum; NaN counts as the maximum
        if W[p, k] == 0.0:
            return 0, 0.0, 0, W
        if p != k:
            W[[k, p]] = W[[p, k]]
            sign = -sign
        piv = W[k, k]
        pm, pe = math.frexp(piv)  # piv = pm * 2^pe exactly
        if pm < 0:
            sign, pm = -sign, -pm
        mant, e2 = math.frexp(mant * pm)  # one rounding, as in det *= pivot
        expo += pe + e2
        if k + 1 < n:
            l = W[k + 1:, k] / piv
            W[k + 1:, k + 1:] = W[k + 1:, k + 1:] - np.outer(l, W[k, k + 1:])
            W[k + 1:, k] = 0.0
    return sign, mant, expo, W


def det_value(sign: int, mant: float, expo: int) -> float:
    """The determinant as a float64 (overflows to +-inf, underflows to 0 like ldexp)."""
    if mant == 0.0:
        return 0.0
    try:
        return sign * math.ldexp(mant, expo)
    except OverflowError:
        return sign * math.inf
