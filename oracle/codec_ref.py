"""Multi-component inputs (double-double, triple-double, quad-double).

TEST INFRASTRUCTURE ONLY: the tests are the only callers.  An entry given as
k doubles stands for their exact sum (every finite double is a dyadic
rational, so ``Fraction(float)`` is exact); its conversion to the library's
number format is that sum rounded once to ``prec_bits``, to nearest with ties
to even (``fraction_ref.round_rne``).  This is the plain definition of what
``mpcg_from_doubles`` computes; an entry with an infinite or NaN component
has no value and is written as +0.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from mpgen import EXP_ZERO, HostCMat, HostPart, limbs_for
from oracle.fraction_ref import round_rne


def exact_sum(components) -> Fraction:
    """The exact value of an entry's components."""
    total = Fraction(0)
    for c in components:
        total += Fraction(float(c))
    return total


def from_doubles_part(comps: np.ndarray, prec_bits: int) -> HostPart:
    """comps: float64 array (ncomp, cols, rows) -> one real component at prec_bits."""
    ncomp, cols, rows = comps.shape
    L = limbs_for(prec_bits)
    sign = np.zeros((cols, rows), np.uint8)
    exp = np.full((cols, rows), EXP_ZERO, np.int32)
    mant = np.zeros((L, cols, rows), np.uint64)
    for c in range(cols):
        for r in range(rows):
            vals = [float(v) for v in comps[:, c, r]]
            if not all(math.isfinite(v) for v in vals):
                continue
            s, e, q = round_rne(exact_sum(vals), prec_bits)
            if q == 0:
                continue
            M = q << (64 * L - prec_bits)
            sign[c, r] = s
            exp[c, r] = e
            for l in range(L):
                mant[l, c, r] = (M >> (64 * l)) & ((1 << 64) - 1)
    return HostPart(rows, cols, rows, L, sign, exp, mant)


def from_doubles(re: np.ndarray, im: np.ndarray, prec_bits: int) -> HostCMat:
    return HostCMat(from_doubles_part(re, prec_bits), from_doubles_part(im, prec_bits))


def round_double(x: Fraction):
    """IEEE binary64 rounding of a rational to nearest, ties to even, with
    gradual underflow and no upper limit: (value as a Fraction, overflow),
    overflow meaning the value reaches 2^1024 (beyond the largest double)."""
    if x == 0:
        return Fraction(0), False
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()  # 2^e <= a < 2^(e+1) after adjusting
    while Fraction(2) ** e > a:
        e -= 1
    while a >= Fraction(2) ** (e + 1):
        e += 1
    ulp_exp = max(e - 52, -1074)
    scaled = a / Fraction(2) ** ulp_exp
    q = scaled.numerator // scaled.denominator
    rem = scaled - q
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and q % 2 == 1):
        q += 1
    v = Fraction(q) * Fraction(2) ** ulp_exp
    return (-v if x < 0 else v), v >= Fraction(2) ** 1024


def to_doubles_part(part: HostPart, prec_bits: int, ncomp: int) -> np.ndarray:
    """Each stored entry as ncomp doubles, greedily: component i is the double
    nearest what the earlier components leave (a zero that underflows keeps
    the remainder's sign, an exactly zero remainder gives +0, beyond the
    largest double +-infinity); float64 array (ncomp, cols, rows)."""
    from oracle.fraction_ref import decode
    out = np.zeros((ncomp, part.cols, part.rows), np.float64)
    for c in range(part.cols):
        for r in range(part.rows):
            rest = decode(part, r, c, prec_bits)
            for i in range(ncomp):
                if rest == 0:
                    out[i, c, r] = 0.0
                    continue
                v, overflow = round_double(rest)
                if overflow:
                    out[i, c, r] = math.inf if rest > 0 else -math.inf
                elif v == 0:
                    out[i, c, r] = 0.0 if rest > 0 else -0.0
                else:
                    out[i, c, r] = float(v)  # exact: v is a double
                rest -= v
    return out


def to_doubles(C: HostCMat, prec_bits: int, ncomp: int):
    return to_doubles_part(C.re, prec_bits, ncomp), to_doubles_part(C.im, prec_bits, ncomp)
