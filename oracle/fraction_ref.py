"""Brute-force rational reference (tiny inputs only).

TEST INFRASTRUCTURE ONLY.  Exact rational evaluation of C = AB with Python's
``fractions.Fraction`` (eq. 2 with the complex product of eq. 3), followed by
the textbook round-to-nearest, ties-to-even rule at ``prec_bits``.  It shares
nothing with ``oracle_cgemm.c`` except the number format it decodes, and is
used to pin that C oracle on small random and hand-made cases.
"""
from __future__ import annotations

from fractions import Fraction

from mpgen import EXP_ZERO, HostCMat, HostPart


def decode(part: HostPart, r: int, c: int, prec_bits: int) -> Fraction:
    """Stored entry -> exact rational, reading only the top prec_bits significand bits."""
    e = int(part.exp[c, r])
    if e == EXP_ZERO:
        return Fraction(0)
    M = 0
    for l in range(part.L - 1, -1, -1):
        M = (M << 64) | int(part.mant[l, c, r])
    drop = 64 * part.L - prec_bits
    M >>= drop  # p-bit integer significand, value = M * 2^(e - p)
    v = Fraction(M) * Fraction(2) ** (e - prec_bits)
    return -v if part.sign[c, r] else v


def round_rne(x: Fraction, prec_bits: int):
    """Textbook RNE of a rational to prec_bits.

    Returns (sign, exp, q) with x ~= (-1)^sign * q * 2^(exp - p), q in
    [2^(p-1), 2^p), or (0, None, 0) for zero."""
    if x == 0:
        return 0, None, 0
    s = 1 if x < 0 else 0
    a = -x if s else x
    # exponent e with 2^(e-1) <= a < 2^e
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** (e - 1) > a:
        e -= 1
    while a >= Fraction(2) ** e:
        e += 1
    scaled = a * Fraction(2) ** (prec_bits - e)  # in [2^(p-1), 2^p)
    q = scaled.numerator // scaled.denominator
    rem = scaled - q
    half = Fraction(1, 2)
    if rem > half or (rem == half and q % 2 == 1):
        q += 1
    if q == 1 << prec_bits:
        q = 1 << (prec_bits - 1)
        e += 1
    return s, e, q


def exact_product(A: HostCMat, B: HostCMat, prec_bits: int):
    """Exact rationals (Re, Im) of every entry of AB, as nested lists [i][j]."""
    m, k, n = A.rows, A.cols, B.cols
    ar = [[decode(A.re, i, t, prec_bits) for t in range(k)] for i in range(m)]
    ai = [[decode(A.im, i, t, prec_bits) for t in range(k)] for i in range(m)]
    br = [[decode(B.re, t, j, prec_bits) for j in range(n)] for t in range(k)]
    bi = [[decode(B.im, t, j, prec_bits) for j in range(n)] for t in range(k)]
    re = [[sum((ar[i][t] * br[t][j] - ai[i][t] * bi[t][j] for t in range(k)), Fraction(0))
           for j in range(n)] for i in range(m)]
    im = [[sum((ar[i][t] * bi[t][j] + ai[i][t] * br[t][j] for t in range(k)), Fraction(0))
           for j in range(n)] for i in range(m)]
    return re, im


def rounded_product(A: HostCMat, B: HostCMat, prec_bits: int):
    """RNE(p) of every entry: nested lists [i][j] of ((s, e, q) Re, (s, e, q) Im)."""
    re, im = exact_product(A, B, prec_bits)
    return [[(round_rne(re[i][j], prec_bits), round_rne(im[i][j], prec_bits))
             for j in range(len(re[0]))] for i in range(len(re))]


def rounded_product_acc(A: HostCMat, B: HostCMat, Cin: HostCMat, prec_bits: int, sign: int):
    """RNE(p) of Cin + sign * AB, entry by entry (one rounding of the exact sum)."""
    re, im = exact_product(A, B, prec_bits)
    out = []
    for i in range(len(re)):
        row = []
        for j in range(len(re[0])):
            cr = decode(Cin.re, i, j, prec_bits)
            ci = decode(Cin.im, i, j, prec_bits)
            row.append((round_rne(cr + sign * re[i][j], prec_bits), round_rne(ci + sign * im[i][j], prec_bits)))
        out.append(row)
    return out


def triple_value(t) -> Fraction:
    """The exact value of a (sign, exp, q) triple from round_rne."""
    s, e, q = t
    if q == 0:
        return Fraction(0)
    v = Fraction(q) * Fraction(2) ** (e - q.bit_length())
    return -v if s else v


def stored_as_triple(part: HostPart, r: int, c: int, prec_bits: int):
    """A stored (output) entry as (sign, exp, q) comparable with round_rne's result."""
    e = int(part.exp[c, r])
    if e == EXP_ZERO:
        return 0, None, 0
    M = 0
    for l in range(part.L - 1, -1, -1):
        M = (M << 64) | int(part.mant[l, c, r])
    drop = 64 * part.L - prec_bits
    assert M & ((1 << drop) - 1) == 0, "bits below the precision must be zero"
    return int(part.sign[c, r]), e, M >> drop
