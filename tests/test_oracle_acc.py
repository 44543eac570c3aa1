"""Pins of the oracle's accumulating product C := Cin + sign * A B (one rounding
of the exact sum), against things other than itself (no GPU needed):

* brute-force rational arithmetic (fractions.Fraction + textbook rounding) on
  tiny random inputs, with the addend shifted from far below to far above the
  product and through exact cancellation;
* Cin = 0 reduces to the plain product, A = 0 returns Cin unchanged;
* sign symmetry: Cin - A B = -((-Cin) + A B);
* exactly representable products cancel to +0.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import fraction_ref as fr
from mpgen import EXP_ZERO, HostCMat, empty_cmat, random_cmat, scale_exponents
from tests.mp_util import cmat_from_values, equal_parts, negate_part, value_of


def _triples(C: HostCMat, p: int, m: int, n: int):
    return [[(fr.stored_as_triple(C.re, i, j, p), fr.stored_as_triple(C.im, i, j, p)) for j in range(n)]
            for i in range(m)]


def _shifted(M: HostCMat, shift: int) -> HostCMat:
    S = M.copy()
    scale_exponents(S.re, rows=slice(None), shift=shift)
    scale_exponents(S.im, rows=slice(None), shift=shift)
    return S


def _neg(M: HostCMat) -> HostCMat:
    return HostCMat(negate_part(M.re), negate_part(M.im))


def _round_to_cmat(vals, p: int, m: int, n: int) -> HostCMat:
    """The rounded product as stored numbers (used as an addend)."""
    re = [[fr.triple_value(vals[i][j][0]) for j in range(n)] for i in range(m)]
    im = [[fr.triple_value(vals[i][j][1]) for j in range(n)] for i in range(m)]
    return cmat_from_values(re, im, p)


@pytest.mark.parametrize("trial", range(48))
def test_acc_bruteforce_random(trial):
    rng = np.random.default_rng(5000 + trial)
    m, n, k = (int(x) for x in rng.integers(1, 4, size=3))
    p = int(rng.choice([2, 3, 8, 53, 64, 65, 128, 200]))
    R = int(rng.choice([0, 4, 20]))
    A = random_cmat([trial], 0, m, k, p, R, zero_frac=0.15)
    B = random_cmat([trial], 1, k, n, p, R, zero_frac=0.15)
    # the addend from far below the product (a signed sticky bit) to far above
    # it (the product only breaks ties), through the overlapping range
    shift = int(rng.choice([-400, -p - 3, -p - 1, -p, -7, -1, 0, 1, 5, p - 1, p + 1, p + 3, 400]))
    Cin = _shifted(random_cmat([trial], 2, m, n, p, R, zero_frac=0.15), shift)
    sign = 1 if trial % 2 == 0 else -1
    ref = fr.rounded_product_acc(A, B, Cin, p, sign)
    for form in (oracle.FORM_4M, oracle.FORM_3M):
        C = oracle.cgemm_acc(A, B, Cin, p, sign, form=form, nthreads=2)
        assert _triples(C, p, m, n) == ref, (trial, form, shift, sign)
        s, e, mm = oracle.cgemm_acc_entries(A, B, Cin, [0, m - 1], [n - 1, 0], p, sign, form=form, nthreads=2)
        for t, (i, j) in enumerate([(0, n - 1), (m - 1, 0)]):
            for comp, part in enumerate((C.re, C.im)):
                assert e[t, comp] == part.exp[j, i]
                if e[t, comp] != EXP_ZERO:
                    assert s[t, comp] == part.sign[j, i] and np.array_equal(mm[t, comp], part.mant[:, j, i])


@pytest.mark.parametrize("p", [2, 7, 53, 64, 130])
def test_acc_cancellation_against_fractions(p):
    """Cin = -RNE(AB): the result is the rounding error of the product, rounded
    once; with sign = -1 and Cin = RNE(AB) the same error with the other sign."""
    m, n, k = 3, 2, 4
    A = random_cmat(91 + p, 0, m, k, p, 6)
    B = random_cmat(91 + p, 1, k, n, p, 6)
    rp = fr.rounded_product(A, B, p)
    Rn = _round_to_cmat(rp, p, m, n)
    for Cin, sign in ((_neg(Rn), 1), (Rn, -1)):
        ref = fr.rounded_product_acc(A, B, Cin, p, sign)
        C = oracle.cgemm_acc(A, B, Cin, p, sign, nthreads=2)
        assert _triples(C, p, m, n) == ref
        # |C| is at most half an ulp of the rounded product
        re, im = fr.exact_product(A, B, p)
        for i in range(m):
            for j in range(n):
                for comp, exact in ((0, re[i][j]), (1, im[i][j])):
                    got = value_of(C.re if comp == 0 else C.im, i, j)
                    r = fr.triple_value(rp[i][j][comp])
                    assert got == 0 or abs(got) <= abs(r) * Fraction(1, 2 ** p), (exact, got)


def test_acc_zero_addend_is_the_product():
    p = 150
    A = random_cmat(3, 0, 5, 7, p, 30, zero_frac=0.1)
    B = random_cmat(3, 1, 7, 4, p, 30, zero_frac=0.1)
    Z = empty_cmat(5, 4, p)
    for form in (oracle.FORM_4M, oracle.FORM_3M):
        C = oracle.cgemm(A, B, p, form=form)
        for sign in (1, -1):
            D = oracle.cgemm_acc(A, B, Z, p, sign, form=form)
            if sign == 1:
                assert equal_parts(D.re, C.re, 5, 4) and equal_parts(D.im, C.im, 5, 4)
            else:
                assert equal_parts(D.re, negate_part(C.re), 5, 4) and equal_parts(D.im, negate_part(C.im), 5, 4)


def test_acc_zero_product_returns_addend():
    p = 97
    A = empty_cmat(4, 6, p)  # all zeros
    B = random_cmat(4, 1, 6, 3, p, 40)
    Cin = random_cmat(4, 2, 4, 3, p, 40, zero_frac=0.2)
    for sign in (1, -1):
        D = oracle.cgemm_acc(A, B, Cin, p, sign)
        assert equal_parts(D.re, Cin.re, 4, 3) and equal_parts(D.im, Cin.im, 4, 3)


@pytest.mark.parametrize("p", [5, 64, 300])
def test_acc_sign_symmetry(p):
    A = random_cmat(8, 0, 4, 5, p, 12)
    B = random_cmat(8, 1, 5, 3, p, 12)
    Cin = random_cmat(8, 2, 4, 3, p, 12)
    D1 = oracle.cgemm_acc(A, B, Cin, p, -1)
    D2 = oracle.cgemm_acc(A, B, _neg(Cin), p, 1)
    assert equal_parts(D1.re, negate_part(D2.re), 4, 3) and equal_parts(D1.im, negate_part(D2.im), 4, 3)


def test_acc_exact_cancellation_gives_plus_zero():
    """Short significands make A B exact in p bits; Cin = A B then cancels."""
    p = 64
    re = [[1, 3], [Fraction(5, 4), -2]]
    im = [[0, Fraction(1, 2)], [-1, 7]]
    A = cmat_from_values(re, im, p)
    B = cmat_from_values([[2, -1], [Fraction(3, 8), 4]], [[1, 0], [Fraction(-1, 2), 5]], p)
    rp = fr.rounded_product(A, B, p)
    P = _round_to_cmat(rp, p, 2, 2)
    D = oracle.cgemm_acc(A, B, P, p, -1)
    assert (D.re.exp[:2, :2] == EXP_ZERO).all() and (D.im.exp[:2, :2] == EXP_ZERO).all()
    assert (D.re.sign[:2, :2] == 0).all() and (D.im.sign[:2, :2] == 0).all()
