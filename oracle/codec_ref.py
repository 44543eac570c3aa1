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
