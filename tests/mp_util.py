"""Test helpers: encode exact dyadic rationals into the stored number format."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from mpgen import EXP_ZERO, HostCMat, HostPart, limbs_for


def encode(value, prec_bits: int):
    """Exact dyadic rational (int, Fraction or (num, pow2)) with at most prec_bits
    significant bits -> (sign, exp, limbs list)."""
    if isinstance(value, tuple):
        num, pw = value
        v = Fraction(num) * Fraction(2) ** pw
    else:
        v = Fraction(value)
    if v == 0:
        return 0, int(EXP_ZERO), [0] * limbs_for(prec_bits)
    s = 1 if v < 0 else 0
    v = abs(v)
    assert v.denominator & (v.denominator - 1) == 0, "not dyadic"
    # v = N * 2^-t with N odd
    t = v.denominator.bit_length() - 1
    N = v.numerator
    tz = (N & -N).bit_length() - 1  # an integer value may carry trailing zero bits
    N >>= tz
    t -= tz
    nb = N.bit_length()
    assert nb <= prec_bits, "too many significant bits"
    e = nb - t  # value = N/2^nb * 2^e, N/2^nb in [1/2, 1)
    L = limbs_for(prec_bits)
    M = N << (64 * L - nb)
    limbs = [(M >> (64 * l)) & ((1 << 64) - 1) for l in range(L)]
    return s, e, limbs


def part_from_values(vals, prec_bits: int) -> HostPart:
    """vals: 2-D list [rows][cols] of exact values."""
    rows, cols = len(vals), len(vals[0])
    L = limbs_for(prec_bits)
    sign = np.zeros((cols, rows), np.uint8)
    exp = np.full((cols, rows), EXP_ZERO, np.int32)
    mant = np.zeros((L, cols, rows), np.uint64)
    for r in range(rows):
        for c in range(cols):
            s, e, limbs = encode(vals[r][c], prec_bits)
            sign[c, r] = s
            exp[c, r] = e
            for l in range(L):
                mant[l, c, r] = limbs[l]
    return HostPart(rows, cols, rows, L, sign, exp, mant)


def cmat_from_values(re_vals, im_vals, prec_bits: int) -> HostCMat:
    return HostCMat(part_from_values(re_vals, prec_bits), part_from_values(im_vals, prec_bits))


def value_of(part: HostPart, r: int, c: int) -> Fraction:
    e = int(part.exp[c, r])
    if e == EXP_ZERO:
        return Fraction(0)
    M = 0
    for l in range(part.L - 1, -1, -1):
        M = (M << 64) | int(part.mant[l, c, r])
    v = Fraction(M) * Fraction(2) ** (e - 64 * part.L)
    return -v if part.sign[c, r] else v


def transpose_part(p: HostPart) -> HostPart:
    """Transpose of a component (rows <-> cols), ld = new rows."""
    R, C = p.rows, p.cols
    sign = np.ascontiguousarray(p.sign[:, :R].T)
    exp = np.ascontiguousarray(p.exp[:, :R].T)
    mant = np.ascontiguousarray(np.transpose(p.mant[:, :, :R], (0, 2, 1)))
    return HostPart(C, R, C, p.L, sign, exp, mant)


def negate_part(p: HostPart) -> HostPart:
    q = p.copy()
    nz = q.exp != EXP_ZERO
    q.sign[nz] ^= 1
    return q


def equal_parts(a: HostPart, b: HostPart, rows: int, cols: int, signed_zero_insensitive: bool = True) -> bool:
    ea, eb = a.exp[:cols, :rows], b.exp[:cols, :rows]
    if not np.array_equal(ea, eb):
        return False
    nz = ea != EXP_ZERO
    if not np.array_equal(a.sign[:cols, :rows][nz], b.sign[:cols, :rows][nz]):
        return False
    return bool(np.array_equal(a.mant[:, :cols, :rows][:, nz], b.mant[:, :cols, :rows][:, nz]))
