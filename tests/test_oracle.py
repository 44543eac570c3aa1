"""Pins of the CPU oracle against things other than itself (no GPU needed).

* brute-force rational arithmetic (fractions.Fraction + textbook rounding) on
  tiny random inputs, both evaluation forms;
* an exhaustive sweep of 1x1x1 complex products at p = 2;
* IEEE binary64 (Python floats, math.fsum) at p = 53;
* mpmath's correctly rounded conversion at larger precisions;
* hand-worked rounding cases (tests/golden/rne_worked_cases.txt);
* algebraic invariants: A I = A, I B = B, (AB)^H = B^H A^H, (AB)^T = B^T A^T,
  power-of-two row scaling, permutations, real inputs, 3M form == 4M form.
"""
from __future__ import annotations

import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import fraction_ref as fr
from mpgen import EXP_ZERO, HostCMat, empty_cmat, random_cmat
from tests.mp_util import (cmat_from_values, equal_parts, negate_part, transpose_part, value_of)

HERE = os.path.dirname(os.path.abspath(__file__))


def _triples(C: HostCMat, p: int, m: int, n: int):
    return [[(fr.stored_as_triple(C.re, i, j, p), fr.stored_as_triple(C.im, i, j, p)) for j in range(n)]
            for i in range(m)]


# ---------------------------------------------------------------------------
# brute force
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("trial", range(60))
def test_bruteforce_random(trial):
    rng = np.random.default_rng(1000 + trial)
    m, n, k = (int(x) for x in rng.integers(1, 5, size=3))
    p = int(rng.choice([2, 3, 7, 8, 53, 64, 65, 127, 128, 256]))
    R = int(rng.choice([0, 3, 20, 70]))
    A = random_cmat([trial], 0, m, k, p, R, zero_frac=0.2)
    B = random_cmat([trial], 1, k, n, p, R, zero_frac=0.2)
    ref = fr.rounded_product(A, B, p)
    for form in (oracle.FORM_4M, oracle.FORM_3M):
        C = oracle.cgemm(A, B, p, form=form, nthreads=2)
        assert _triples(C, p, m, n) == ref


def test_bruteforce_hypothesis():
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=60, deadline=None, derandomize=True)
    @hyp.given(m=st.integers(1, 4), n=st.integers(1, 4), k=st.integers(1, 4),
               p=st.sampled_from([2, 3, 8, 53, 64, 65, 128, 200]), R=st.integers(0, 70),
               seed=st.integers(0, 2 ** 31), zf=st.sampled_from([0.0, 0.3]))
    def check(m, n, k, p, R, seed, zf):
        A = random_cmat([seed], 0, m, k, p, R, zero_frac=zf)
        B = random_cmat([seed], 1, k, n, p, R, zero_frac=zf)
        C = oracle.cgemm(A, B, p, nthreads=1)
        assert _triples(C, p, m, n) == fr.rounded_product(A, B, p)

    check()


def _rne_int(num: int, pw: int, p: int):
    """Textbook RNE of num * 2^pw on integers -> (sign, exp, q) or (0, None, 0)."""
    if num == 0:
        return 0, None, 0
    s = 1 if num < 0 else 0
    a = -num if s else num
    nb = a.bit_length()
    e = nb + pw
    if nb <= p:
        return s, e, a << (p - nb)
    sh = nb - p
    q = a >> sh
    rem = a & ((1 << sh) - 1)
    half = 1 << (sh - 1)
    if rem > half or (rem == half and q & 1):
        q += 1
    if q == 1 << p:
        q >>= 1
        e += 1
    return s, e, q


def test_exhaustive_1x1x1_p2():
    """Every 1x1x1 complex product of p = 2 numbers with exponents in [-2, 2] (and zero)."""
    p = 2
    vals = [Fraction(0)]
    for sgn in (1, -1):
        for sig in (2, 3):  # p-bit significands
            for e in range(-2, 3):
                vals.append(sgn * Fraction(sig, 4) * Fraction(2) ** e)
    nv = len(vals)  # 21
    pairs = [(a, b) for a in vals for b in vals]  # (re, im) of one complex number
    m = n = len(pairs)
    A = cmat_from_values([[pr[0]] for pr in pairs], [[pr[1]] for pr in pairs], p)
    B = cmat_from_values([[pr[0] for pr in pairs]], [[pr[1] for pr in pairs]], p)
    C = oracle.cgemm(A, B, p)
    # expected on integers: every value is an integer multiple of 2^-4
    ints = [int(v * 16) for v in vals]
    idx = {v: t for t, v in enumerate(vals)}
    bad = 0
    for i, (ar, ai) in enumerate(pairs):
        iar, iai = ints[idx[ar]], ints[idx[ai]]
        for j, (br, bi) in enumerate(pairs):
            ibr, ibi = ints[idx[br]], ints[idx[bi]]
            er = _rne_int(iar * ibr - iai * ibi, -8, p)
            ei = _rne_int(iar * ibi + iai * ibr, -8, p)
            if (fr.stored_as_triple(C.re, i, j, p), fr.stored_as_triple(C.im, i, j, p)) != (er, ei):
                bad += 1
    assert nv == 21 and bad == 0


# ---------------------------------------------------------------------------
# library pins
# ---------------------------------------------------------------------------
def _random_short(rng, rows, cols, bits, p, erange):
    """Values with `bits`-bit significands (exactly representable at p)."""
    out = []
    for _ in range(rows):
        row = []
        for _ in range(cols):
            sig = int(rng.integers(1 << (bits - 1), 1 << bits))
            e = int(rng.integers(-erange, erange + 1))
            s = -1 if rng.integers(0, 2) else 1
            row.append(s * Fraction(sig) * Fraction(2) ** (e - bits))
        out.append(row)
    return out


def _to_float(part, r, c):
    return float(value_of(part, r, c))


def test_p53_real_products_match_ieee():
    """Im = 0, p = 53: a 1x1x1 product is one IEEE multiplication."""
    rng = np.random.default_rng(53)
    av = _random_short(rng, 200, 1, 53, 53, 40)
    bv = _random_short(rng, 1, 200, 53, 53, 40)
    zeros_a = [[0] for _ in range(200)]
    zeros_b = [[0] * 200]
    A = cmat_from_values(av, zeros_a, 53)
    B = cmat_from_values(bv, zeros_b, 53)
    C = oracle.cgemm(A, B, 53)
    for i in range(0, 200, 7):
        for j in range(0, 200, 3):
            assert _to_float(C.re, i, j) == float(av[i][0]) * float(bv[0][j])
            assert C.im.exp[j, i] == EXP_ZERO


def test_p53_complex_sums_match_fsum():
    """p = 53 with 26-bit inputs: every product is exact in binary64 and math.fsum
    returns the correctly rounded sum, so Re and Im must equal fsum of the terms."""
    rng = np.random.default_rng(26)
    m, n, k = 6, 5, 40
    ar = _random_short(rng, m, k, 26, 53, 30)
    ai = _random_short(rng, m, k, 26, 53, 30)
    br = _random_short(rng, k, n, 26, 53, 30)
    bi = _random_short(rng, k, n, 26, 53, 30)
    A = cmat_from_values(ar, ai, 53)
    B = cmat_from_values(br, bi, 53)
    for form in (oracle.FORM_4M, oracle.FORM_3M):
        C = oracle.cgemm(A, B, 53, form=form)
        for i in range(m):
            for j in range(n):
                re_terms, im_terms = [], []
                for t in range(k):
                    re_terms += [float(ar[i][t]) * float(br[t][j]), -(float(ai[i][t]) * float(bi[t][j]))]
                    im_terms += [float(ar[i][t]) * float(bi[t][j]), float(ai[i][t]) * float(br[t][j])]
                assert _to_float(C.re, i, j) == math.fsum(re_terms)
                assert _to_float(C.im, i, j) == math.fsum(im_terms)


@pytest.mark.parametrize("p", [64, 113, 256, 512])
def test_mpmath_correct_rounding(p):
    mpmath = pytest.importorskip("mpmath")
    A = random_cmat(p, 0, 3, 5, p, 12)
    B = random_cmat(p, 1, 5, 4, p, 12)
    C = oracle.cgemm(A, B, p)
    ctx = mpmath.mp.clone()
    for i in range(3):
        for j in range(4):
            for comp, part in ((0, C.re), (1, C.im)):
                # exact value from mpmath at a working precision that holds it exactly
                ctx.prec = 4 * p + 400
                acc = ctx.mpf(0)
                for t in range(5):
                    a = (ctx.mpf(value_of(A.re, i, t).numerator) / value_of(A.re, i, t).denominator,
                         ctx.mpf(value_of(A.im, i, t).numerator) / value_of(A.im, i, t).denominator)
                    b = (ctx.mpf(value_of(B.re, t, j).numerator) / value_of(B.re, t, j).denominator,
                         ctx.mpf(value_of(B.im, t, j).numerator) / value_of(B.im, t, j).denominator)
                    acc += (a[0] * b[0] - a[1] * b[1]) if comp == 0 else (a[0] * b[1] + a[1] * b[0])
                ctx.prec = p
                rounded = +acc  # round to nearest, ties to even
                got = value_of(part, i, j)
                sgn, man, ex, _bc = rounded._mpf_  # value = (-1)^sgn * man * 2^ex
                want = Fraction(int(man)) * Fraction(2) ** int(ex) if man else Fraction(0)
                want = -want if sgn else want
                assert want == got


# ---------------------------------------------------------------------------
# worked rounding cases
# ---------------------------------------------------------------------------
def _parse_golden():
    cases = []
    with open(os.path.join(HERE, "golden", "rne_worked_cases.txt")) as f:
        for line in f:
            if not line.strip() or line.lstrip().startswith("#"):
                continue
            name, precs, terms, expected, _why = [x.strip() for x in line.split("|")]
            for p in (int(x) for x in precs.split(",")):
                cases.append((name, p, terms, expected))
    return cases


def _ev(expr: str, p: int) -> int:
    return int(eval(expr.replace("^", "**"), {"p": p}))


@pytest.mark.parametrize("name,p,terms,expected", _parse_golden())
def test_worked_rounding_cases(name, p, terms, expected):
    vals = []
    for sgn, num, pw in re.findall(r"\(([+-]),([^,]+),([^)]+)\)", terms):
        v = Fraction(_ev(num, p)) * Fraction(2) ** _ev(pw, p)
        vals.append(-v if sgn == "-" else v)
    k = len(vals)
    A = cmat_from_values([vals], [[0] * k], p)
    B = cmat_from_values([[1] for _ in range(k)], [[0] for _ in range(k)], p)
    C = oracle.cgemm(A, B, p)
    got = fr.stored_as_triple(C.re, 0, 0, p)
    if expected == "zero":
        assert got == (0, None, 0)
    else:
        s, q, e = [x.strip() for x in expected.strip("()").split(",")]
        assert got == (int(s), _ev(e, p), _ev(q, p)), name  # stored_as_triple gives (sign, exp, q)
    assert C.im.exp[0, 0] == EXP_ZERO


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
def _identity(nn: int, p: int) -> HostCMat:
    I = empty_cmat(nn, nn, p)
    for t in range(nn):
        I.re.exp[t, t] = 1  # 1 = 0.5 * 2^1
        I.re.mant[I.L - 1, t, t] = np.uint64(1 << 63)
    return I


@pytest.mark.parametrize("p", [2, 64, 130, 512])
def test_identity(p):
    A = random_cmat(7, 0, 9, 6, p, 30, zero_frac=0.1)
    C = oracle.cgemm(A, _identity(6, p), p)
    assert equal_parts(C.re, A.re, 9, 6) and equal_parts(C.im, A.im, 9, 6)
    B = random_cmat(7, 1, 6, 5, p, 30, zero_frac=0.1)
    C = oracle.cgemm(_identity(6, p), B, p)
    assert equal_parts(C.re, B.re, 6, 5) and equal_parts(C.im, B.im, 6, 5)


def _conj_transpose(M: HostCMat) -> HostCMat:
    return HostCMat(transpose_part(M.re), negate_part(transpose_part(M.im)))


def _transpose(M: HostCMat) -> HostCMat:
    return HostCMat(transpose_part(M.re), transpose_part(M.im))


@pytest.mark.parametrize("p", [3, 100, 256])
def test_conjugate_transpose(p):
    A = random_cmat(17, 0, 5, 7, p, 25)
    B = random_cmat(17, 1, 7, 4, p, 25)
    C = oracle.cgemm(A, B, p)
    D = oracle.cgemm(_conj_transpose(B), _conj_transpose(A), p)  # = (AB)^H
    Ch = _conj_transpose(C)
    assert equal_parts(D.re, Ch.re, 4, 5) and equal_parts(D.im, Ch.im, 4, 5)
    T = oracle.cgemm(_transpose(B), _transpose(A), p)  # = (AB)^T
    Ct = _transpose(C)
    assert equal_parts(T.re, Ct.re, 4, 5) and equal_parts(T.im, Ct.im, 4, 5)


def test_row_scaling_and_permutation():
    p = 96
    A = random_cmat(23, 0, 6, 8, p, 10)
    B = random_cmat(23, 1, 8, 5, p, 10)
    C = oracle.cgemm(A, B, p)
    # diag(2^t) A: row i of C shifts its exponent by t_i, significands unchanged
    t = np.array([0, 60, -7, 3, 1000, -1000], np.int32)
    As = A.copy()
    for part in (As.re, As.im):
        nz = part.exp != EXP_ZERO
        part.exp[:] = np.where(nz, part.exp + t[None, :], part.exp)
    Cs = oracle.cgemm(As, B, p)
    for part, ref in ((Cs.re, C.re), (Cs.im, C.im)):
        nz = ref.exp != EXP_ZERO
        assert np.array_equal(part.exp, np.where(nz, ref.exp + t[None, :], ref.exp))
        assert np.array_equal(part.mant, ref.mant) and np.array_equal(part.sign, ref.sign)
    # permuting the rows of A and the columns of B permutes C
    pr = np.array([3, 0, 5, 1, 4, 2])
    pc = np.array([4, 2, 0, 3, 1])
    Ap = A.copy()
    Bp = B.copy()
    for dst, src in ((Ap.re, A.re), (Ap.im, A.im)):
        dst.sign[:] = src.sign[:, pr]; dst.exp[:] = src.exp[:, pr]; dst.mant[:] = src.mant[:, :, pr]
    for dst, src in ((Bp.re, B.re), (Bp.im, B.im)):
        dst.sign[:] = src.sign[pc]; dst.exp[:] = src.exp[pc]; dst.mant[:] = src.mant[:, pc]
    Cp = oracle.cgemm(Ap, Bp, p)
    for part, ref in ((Cp.re, C.re), (Cp.im, C.im)):
        assert np.array_equal(part.exp, ref.exp[pc][:, pr])
        assert np.array_equal(part.mant, ref.mant[:, pc][:, :, pr])


def test_real_inputs_reduce_to_real_gemm():
    p = 80
    A = random_cmat(31, 0, 5, 6, p, 8)
    B = random_cmat(31, 1, 6, 4, p, 8)
    for M in (A, B):
        M.im.exp[:] = EXP_ZERO
        M.im.mant[:] = 0
    C = oracle.cgemm(A, B, p)
    assert (C.im.exp == EXP_ZERO).all()
    ref = fr.rounded_product(A, B, p)
    assert _triples(C, p, 5, 4) == ref


@pytest.mark.parametrize("seed", range(4))
def test_3m_form_equals_4m_form(seed):
    p = [64, 200, 512, 1024][seed]
    A = random_cmat(40 + seed, 0, 7, 9, p, 40, zero_frac=0.1)
    B = random_cmat(40 + seed, 1, 9, 6, p, 40, zero_frac=0.1)
    C4 = oracle.cgemm(A, B, p, form=oracle.FORM_4M)
    C3 = oracle.cgemm(A, B, p, form=oracle.FORM_3M)
    assert equal_parts(C4.re, C3.re, 7, 6) and equal_parts(C4.im, C3.im, 7, 6)
    for i in range(0, 7, 3):
        for j in range(0, 6, 2):
            assert oracle.exact_entry(A, B, i, j, 1, p, oracle.FORM_4M) == \
                   oracle.exact_entry(A, B, i, j, 1, p, oracle.FORM_3M) or \
                   Fraction(*_frac(oracle.exact_entry(A, B, i, j, 1, p, oracle.FORM_4M))) == \
                   Fraction(*_frac(oracle.exact_entry(A, B, i, j, 1, p, oracle.FORM_3M)))


def _frac(ne):
    num, e = ne
    return (num * 2 ** e, 1) if e >= 0 else (num, 2 ** (-e))


def test_exact_entry_matches_fractions():
    p = 70
    A = random_cmat(9, 0, 3, 6, p, 50, zero_frac=0.2)
    B = random_cmat(9, 1, 6, 3, p, 50, zero_frac=0.2)
    re_, im_ = fr.exact_product(A, B, p)
    for i in range(3):
        for j in range(3):
            for comp, ref in ((0, re_[i][j]), (1, im_[i][j])):
                num, e = oracle.exact_entry(A, B, i, j, comp, p)
                assert Fraction(*_frac((num, e))) == ref


def test_entries_api_matches_full():
    p = 128
    A = random_cmat(12, 0, 10, 11, p, 9)
    B = random_cmat(12, 1, 11, 8, p, 9)
    C = oracle.cgemm(A, B, p)
    rows = np.array([0, 9, 4, 4, 7])
    cols = np.array([0, 7, 3, 5, 0])
    s, e, mm = oracle.cgemm_entries(A, B, rows, cols, p)
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((C.re, C.im)):
            assert e[t, comp] == part.exp[j, i]
            if e[t, comp] != EXP_ZERO:
                assert s[t, comp] == part.sign[j, i]
                assert np.array_equal(mm[t, comp], part.mant[:, j, i])


def test_low_bits_below_precision_are_ignored():
    p = 100
    A = random_cmat(2, 0, 4, 5, p, 6)
    B = random_cmat(2, 1, 5, 3, p, 6)
    C = oracle.cgemm(A, B, p)
    A2 = A.copy()
    A2.re.mant[0] |= np.uint64((1 << 28) - 1)  # 64*2 - 100 = 28 ignored bits
    C2 = oracle.cgemm(A2, B, p)
    assert equal_parts(C.re, C2.re, 4, 3) and equal_parts(C.im, C2.im, 4, 3)
