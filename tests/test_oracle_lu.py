"""Pins of the LU oracle (oracle/lu_ref.py) against things other than itself
(no GPU needed):

* the reciprocal (each component of 1/y rounded once, as MPC divides) agrees
  with mpmath's division at a working precision far above 3p rounded to p,
  and at p = 53 with IEEE double division 1.0 / y for real and imaginary y;
  it is exact for +-2^t, +-i 2^t and 2^t (1 +- i); conjugating y conjugates
  it, multiplying y by i multiplies it by -i, and scaling y by 2^3 scales it
  by 2^-3, bit for bit;
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


def _pivots(p, count, seed, R=6):
    """Random 1 x 1 pivots; every third purely real or purely imaginary, and a
    few with parts far apart in magnitude."""
    out = []
    for t in range(count):
        y = random_cmat([41, seed, p, t], 0, 1, 1, p, R)
        if t % 3 == 0:
            part = y.im if t % 2 == 0 else y.re
            part.exp[...] = np.iinfo(np.int32).min
        elif t % 5 == 1:
            y.im.exp[...] += (3 * p + t) * (1 if t % 2 else -1)  # around and beyond 3p bits apart
        out.append(y)
    return out


def _mp_round(num, den, p):
    """RNE_p(num / den) through mpmath: the quotient at a working precision
    far above 3p (so no rounding boundary can lie between it and the exact
    value), then rounded to p bits by mpmath."""
    import mpmath
    if num == 0:
        return Fraction(0)
    with mpmath.workprec(8 * p + 400):
        q = mpmath.mpf(num.numerator) / mpmath.mpf(num.denominator) * mpmath.mpf(den.denominator) / \
            mpmath.mpf(den.numerator)
    with mpmath.workprec(p):
        r = +q
    sign, man, exp, _ = r._mpf_  # read without converting (a conversion rounds at the default precision)
    v = Fraction(int(man)) * Fraction(2) ** int(exp)
    return -v if sign else v


@pytest.mark.parametrize("p", [2, 3, 53, 64, 65, 128, 256, 1000])
def test_reciprocal_matches_mpmath(p):
    for y in _pivots(p, 15, 1):
        yv = _val(y, 0, 0, p)
        d = yv[0] * yv[0] + yv[1] * yv[1]
        r = _val(lu_ref.reciprocal(y, p), 0, 0, p)
        assert r == (_mp_round(yv[0], d, p), _mp_round(-yv[1], d, p)), p


def test_reciprocal_p53_real_and_imaginary_match_ieee_division():
    rng = np.random.default_rng(45)
    p = 53
    for t in range(400):
        x = float(rng.uniform(0.5, 1.0)) * 2.0 ** int(rng.integers(-60, 61)) * (1 if t % 2 else -1)
        fx = Fraction(x)
        if t % 4 < 2:   # y = x real: 1/y = 1/x
            y, want = to_cmat([[(fx, Fraction(0))]], p), (Fraction(1.0 / x), Fraction(0))
        else:           # y = i x: 1/y = -i / x
            y, want = to_cmat([[(Fraction(0), fx)]], p), (Fraction(0), Fraction(-1.0 / x))
        assert _val(lu_ref.reciprocal(y, p), 0, 0, p) == want, x


@pytest.mark.parametrize("p", [2, 64, 256])
def test_reciprocal_symmetries(p):
    for y in _pivots(p, 12, 2):
        yr, yi = _val(y, 0, 0, p)
        r = _val(lu_ref.reciprocal(y, p), 0, 0, p)
        rc = _val(lu_ref.reciprocal(to_cmat([[(yr, -yi)]], p), p), 0, 0, p)
        assert rc == (r[0], -r[1])                       # 1/conj(y) = conj(1/y)
        ri = _val(lu_ref.reciprocal(to_cmat([[(-yi, yr)]], p), p), 0, 0, p)
        assert ri == (r[1], -r[0])                       # 1/(i y) = -i / y
        r8 = _val(lu_ref.reciprocal(to_cmat([[(yr * 8, yi * 8)]], p), p), 0, 0, p)
        assert r8 == (r[0] / 8, r[1] / 8)                # 1/(8 y) = (1/y) / 8


@pytest.mark.parametrize("p", [2, 64, 256])
def test_reciprocal_of_powers_of_two_is_exact(p):
    for t in (-5, 0, 3):
        for re, im in ((1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, 1)):
            y = to_cmat([[(Fraction(re) * Fraction(2) ** t, Fraction(im) * Fraction(2) ** t)]], p)
            r = _val(lu_ref.reciprocal(y, p), 0, 0, p)
            assert r == _recip_exact((Fraction(re) * Fraction(2) ** t, Fraction(im) * Fraction(2) ** t))


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
