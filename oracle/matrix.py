"""Matrix product and the product postcondition of the oracle.

Section 3.4: matrices are stored as one row-major array and provide multiply (matrix by
matrix).  The product postcondition is a Freivalds-style check: for seeded vectors r_k,
e = C r - A (B r) is compared row by row against the a-priori rounding bound of a float32
product, gamma * |A| (|B| |r|), with gamma = 2Ku / (1 - 2Ku), K the inner dimension and
u = 2^-24, plus 2^-40 slack for the float64 evaluation of the check itself.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24


def gamma(k: int) -> float:
    """gamma_{2K} = 2Ku / (1 - 2Ku): twice Higham's gamma_K for a length-K float32 dot
    product, since the matrix cores' internal summation order is not specified."""
    t = 2.0 * k * U32
    return t / (1.0 - t)


def matmul64(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A B with float32 entries widened to float64: every product is exact in float64
    and the K-term sums carry float64 rounding only."""
    return np.asarray(A, np.float64) @ np.asarray(B, np.float64)


def matmul_bound(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """|A| |B| in float64, the elementwise scale of the float32 product's rounding error."""
    return np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64))


def product_check(C: np.ndarray, A: np.ndarray, B: np.ndarray, R: np.ndarray):
    """Evaluate the product postcondition.

    R holds one vector per row (nvec x N).  Returns (holds, first_index, measure) where
    first_index is the first violating row, taking the vectors in order and then the rows,
    and measure = max_k,i |e_i| / b_i (0 where b_i = 0 and e_i = 0)."""
    A64 = np.asarray(A, np.float64)
    B64 = np.asarray(B, np.float64)
    C64 = np.asarray(C, np.float64)
    K = A64.shape[1]
    tol = gamma(K) + 2.0 ** -40
    absA, absB = np.abs(A64), np.abs(B64)
    first = -1
    measure = 0.0
    for r in np.asarray(R, np.float64):
        e = C64 @ r - A64 @ (B64 @ r)
        b = absA @ (absB @ np.abs(r))
        bad = ~(np.abs(e) <= tol * b)  # NaN fails
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(b > 0, np.abs(e) / np.where(b > 0, b, 1.0),
                             np.where(e == 0, 0.0, np.inf))
        measure = max(measure, float(np.max(ratio))) if ratio.size else measure
        if first < 0 and np.any(bad):
            first = int(np.nonzero(bad)[0][0])
    return first < 0, first, measure
