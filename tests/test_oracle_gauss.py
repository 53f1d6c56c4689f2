"""Pins of the Gaussian-elimination determinant oracle: closed forms (triangular, diagonal,
permutation matrices), exact rational determinants of small integer matrices, numpy's LAPACK
determinant on random matrices, singular matrices, and exponents beyond float64's range."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle.gauss import det_value, gauss_det


def exact_det(M) -> Fraction:
    """Leibniz formula over exact rationals (small n only)."""
    n = len(M)
    tot = Fraction(0)
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = Fraction(1)
        for i in range(n):
            term *= Fraction(float(M[i][perm[i]]))
        tot += -term if inv % 2 else term
    return tot


def test_triangular_and_diagonal_closed_forms():
    g = np.random.Generator(np.random.PCG64(1))
    for n in (1, 2, 5, 9):
        d = g.integers(1, 9, n) * np.where(g.random(n) < 0.5, -1, 1)
        U = np.triu(g.integers(-5, 6, (n, n)).astype(np.float64), 1) + np.diag(d)
        s, m, e, _ = gauss_det(U.astype(np.float32))
        assert det_value(s, m, e) == float(np.prod(d))  # no pivoting needed, exact products
    s, m, e, _ = gauss_det(np.zeros((0, 0), np.float32))
    assert det_value(s, m, e) == 1.0


def test_permutation_matrices_give_their_sign():
    for seed in range(6):
        n = 3 + seed * 7
        P, perm = W.permutation_matrix_f32(n, seed)
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        s, m, e, _ = gauss_det(P)
        assert det_value(s, m, e) == (-1.0 if inv % 2 else 1.0)


@pytest.mark.parametrize("seed", range(10))
def test_small_integer_matrices_vs_exact(seed):
    g = np.random.Generator(np.random.PCG64(10 + seed))
    n = int(g.integers(1, 7))
    A = g.integers(-6, 7, (n, n)).astype(np.float32)
    ex = exact_det(A)
    got = det_value(*gauss_det(A)[:3])
    if ex == 0:
        assert abs(got) <= 1e-9 * max(1.0, float(np.prod(np.abs(A).sum(axis=1))))
    else:
        assert abs(Fraction(got) - ex) <= abs(ex) * Fraction(1, 10**9)


def test_random_matrices_vs_lapack():
    for n in (4, 50, 200):
        A = W.normal_f32(n * n, 3 + n).reshape(n, n)
        s, m, e, _ = gauss_det(A)
        sl, ld = np.linalg.slogdet(A.astype(np.float64))
        assert s == int(sl)
        assert abs((math.log(m) + e * math.log(2.0)) - ld) <= 1e-10 * max(1.0, abs(ld))


def test_singular_and_huge():
    A = W.normal_f32(36, 4).reshape(6, 6)
    A[4] = A[1]  # two equal rows: elimination makes a zero row exactly
    s, m, e, _ = gauss_det(A)
    assert (s, m, e) == (0, 0.0, 0)
    D = np.diag(np.full(10, 2.0 ** 120)).astype(np.float32)  # det = 2^1200, beyond float64
    s, m, e, _ = gauss_det(D)
    assert (s, m, e) == (1, 0.5, 1201) and det_value(s, m, e) == math.inf
    D[3, 3] = -(2.0 ** -140)  # a subnormal float32 pivot: det = -2^940
    s, m, e, _ = gauss_det(D)
    assert (s, m, e) == (-1, 0.5, 941)
    with pytest.raises(ValueError):
        gauss_det(np.zeros((2, 3), np.float32))
