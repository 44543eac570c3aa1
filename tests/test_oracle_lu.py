"""Pins of the LU oracle (oracle/lu_ref.py) against things other than itself
(no GPU needed):

* the reciprocal is within 2^(3-p) |1/y| of the exact 1/y (Fractions) in each
  component, and exact for +-2^t and +-i 2^t; the seed is within 2^-62 of 1/d;
* matrices built as P^T L U with closed-form factors (tests/lu_cases.py) come
  back as exactly L, U and the interchanges that undo P, for every block
  width, and the solve returns the exact x_k = k + k i;
* on random matrices the factors satisfy the backward-error bound
  |P A - L U| <= 2^(10-p) |L| |U| entrywise (|.| = |Re| + |Im|, exact
  rationals), the multipliers stay bounded, and the solve of the paper's
  problem (b = A x, x_k = k + k i) has a tiny relative error;
* ties between equal pivot keys go to the first row, and a zero pivot column
  is reported as LAPACK's info.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
from mpgen import random_cmat
from oracle import lu_ref
from oracle.fraction_ref import decode
from tests.lu_cases import column, exact_case, to_cmat


def _val(M, r, c, p):
    return decode(M.re, r, c, p), decode(M.im, r, c, p)


def _n1(z):
    return abs(z[0]) + abs(z[1])


def _recip_exact(y):
    d = y[0] * y[0] + y[1] * y[1]
    return y[0] / d, -y[1] / d


@pytest.mark.parametrize("p", [2, 53, 64, 65, 128, 256, 1000])
def test_reciprocal_accuracy(p):
    for seed in range(12):
        y = random_cmat([41, seed, p], 0, 1, 1, p, 6)
        if seed % 3 == 0:  # a purely real or purely imaginary pivot
            part = y.im if seed % 2 == 0 else y.re
            part.exp[...] = np.iinfo(np.int32).min
        yv = _val(y, 0, 0, p)
        r = _val(lu_ref.reciprocal(y, p), 0, 0, p)
        ex = _recip_exact(yv)
        mag = _n1(ex)
        bound = Fraction(2) ** (3 - p) * mag if p >= 64 else Fraction(2) ** (3 - p) * mag * 2
        assert abs(r[0] - ex[0]) <= bound and abs(r[1] - ex[1]) <= bound, (p, seed)


@pytest.mark.parametrize("p", [2, 64, 256])
def test_reciprocal_of_powers_of_two_is_exact(p):
    for t in (-5, 0, 3):
        for re, im in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            y = to_cmat([[(Fraction(re) * Fraction(2) ** t, Fraction(im) * Fraction(2) ** t)]], p)
            r = _val(lu_ref.reciprocal(y, p), 0, 0, p)
            assert r == _recip_exact((Fraction(re) * Fraction(2) ** t, Fraction(im) * Fraction(2) ** t))


def test_seed_accuracy():
    p = 256
    for seed in range(40):
        d = random_cmat([42, seed], 0, 1, 1, p, 40)
        d.im.exp[...] = np.iinfo(np.int32).min
        dv = decode(d.re, 0, 0, p)
        x = decode(lu_ref.seed(d, p).re, 0, 0, p)
        assert abs(x * dv - 1) <= Fraction(1, 2 ** 62)


@pytest.mark.parametrize("n,nb", [(1, 1), (2, 1), (7, 3), (12, 1), (12, 4), (12, 5), (12, 12), (12, 64)])
def test_exact_factors(n, nb):
    p = 256
    case = exact_case(n, seed=n * 10 + nb)
    A = to_cmat(case["A"], p)
    LU, ipiv, info = lu_ref.getrf(A, nb, p)
    assert info == 0
    assert np.array_equal(ipiv, case["ipiv"])
    for i in range(n):
        for j in range(n):
            assert _val(LU, i, j, p) == case["packed"][i][j], (i, j)
    X = lu_ref.getrs(LU, ipiv, to_cmat(column(case["b"]), p), p)
    assert [_val(X, i, 0, p) for i in range(n)] == case["x"]


def _cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


@pytest.mark.parametrize("n,nb,p", [(9, 4, 64), (10, 3, 128), (8, 8, 200)])
def test_backward_error(n, nb, p):
    A = random_cmat([43, n, p], 0, n, n, p, 2)
    LU, ipiv, info = lu_ref.getrf(A, nb, p)
    assert info == 0
    assert all(c <= ipiv[c] < n for c in range(n))
    rows = [[_val(A, i, j, p) for j in range(n)] for i in range(n)]
    for c in range(n):
        rows[c], rows[int(ipiv[c])] = rows[int(ipiv[c])], rows[c]
    F = [[_val(LU, i, j, p) for j in range(n)] for i in range(n)]
    one, zero = (Fraction(1), Fraction(0)), (Fraction(0), Fraction(0))
    Lm = [[F[i][j] if i > j else (one if i == j else zero) for j in range(n)] for i in range(n)]
    Um = [[F[i][j] if i <= j else zero for j in range(n)] for i in range(n)]
    tol = Fraction(2) ** (10 - p)
    for i in range(n):
        for j in range(i):
            assert _n1(Lm[i][j]) <= 2 + tol  # multipliers of partial pivoting by |Re| + |Im|
        for j in range(n):
            acc, mag = zero, Fraction(0)
            for k in range(n):
                t = _cmul(Lm[i][k], Um[k][j])
                acc = (acc[0] + t[0], acc[1] + t[1])
                mag += _n1(Lm[i][k]) * _n1(Um[k][j])
            res = (rows[i][j][0] - acc[0], rows[i][j][1] - acc[1])
            assert _n1(res) <= tol * mag, (i, j)


@pytest.mark.parametrize("n,nb,p", [(16, 5, 256), (12, 12, 128)])
def test_solve_paper_problem(n, nb, p):
    """b = A x rounded at p bits with x_k = k + k i; the computed x has a
    relative error of a few units of 2^-p times the (modest) condition."""
    A = random_cmat([44, n, p], 0, n, n, p, 2)
    x = [(Fraction(k + 1), Fraction(k + 1)) for k in range(n)]
    b = oracle.cgemm(A, to_cmat(column(x), p), p)
    LU, ipiv, info = lu_ref.getrf(A, nb, p)
    X = lu_ref.getrs(LU, ipiv, b, p)
    err = max(_n1((_val(X, k, 0, p)[0] - x[k][0], _val(X, k, 0, p)[1] - x[k][1])) / _n1(x[k]) for k in range(n))
    assert err < Fraction(2) ** (24 - p)


def test_pivot_ties_take_the_first_row():
    p = 64
    one, zero = Fraction(1), Fraction(0)
    # column 0: keys 1/2, 1, 1, 1 -> row 1 (the first of the equal keys)
    vals = [[(Fraction(1, 2), zero), (zero, zero), (zero, zero), (one, zero)],
            [(zero, one), (one, zero), (zero, zero), (zero, zero)],
            [(-one, zero), (zero, zero), (one, zero), (zero, zero)],
            [(zero, -one), (zero, zero), (zero, zero), (zero, one)]]
    LU, ipiv, info = lu_ref.getrf(to_cmat(vals, p), 2, p)
    assert ipiv[0] == 1 and info == 0


def test_zero_pivot_is_reported():
    p = 64
    one, zero = Fraction(1), Fraction(0)
    vals = [[(one, zero), (zero, zero), (one, one)],
            [(Fraction(1, 2), zero), (zero, zero), (zero, one)],
            [(zero, one), (zero, zero), (one, zero)]]
    LU, ipiv, info = lu_ref.getrf(to_cmat(vals, p), 2, p)
    assert info == 2  # column 1 has no nonzero pivot
