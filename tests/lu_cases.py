"""Matrices for the LU tests whose factors are known in closed form.

A = P^T L U with L unit lower (off-diagonal entries (a + b i)/16, |a| + |b| <= 6,
so every multiplier has |Re| + |Im| < 1), U upper with pivots +-2^t or +-i 2^t
(exact reciprocals) and short dyadic entries above the diagonal, and P a
seeded permutation of the rows.  Partial pivoting by |Re| + |Im| then picks,
at every column, the row that holds that row of L U (its key is |u_cc|_1; the
others' are |l u_cc|_1 < |u_cc|_1), every step is exact at 256 bits, and the
factorization returns L and U themselves with the interchanges that undo P.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from tests.mp_util import cmat_from_values


def _cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def exact_case(n: int, seed: int):
    rng = np.random.default_rng([seed, 77])
    zero = (Fraction(0), Fraction(0))
    Lm = [[zero] * n for _ in range(n)]
    Um = [[zero] * n for _ in range(n)]
    for i in range(n):
        Lm[i][i] = (Fraction(1), Fraction(0))
        for j in range(i):
            while True:
                a, b = (int(v) for v in rng.integers(-3, 4, 2))
                if abs(a) + abs(b) <= 6:
                    break
            Lm[i][j] = (Fraction(a, 16), Fraction(b, 16))
        t = int(rng.integers(-3, 4))
        s = 1 if rng.random() < 0.5 else -1
        Um[i][i] = (Fraction(s) * Fraction(2) ** t, Fraction(0)) if rng.random() < 0.5 else \
            (Fraction(0), Fraction(s) * Fraction(2) ** t)
        for j in range(i + 1, n):
            a, b = (int(v) for v in rng.integers(-8, 9, 2))
            Um[i][j] = (Fraction(a, 8), Fraction(b, 8))
    LU = [[zero] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            acc = zero
            for k in range(min(i, j) + 1):
                t = _cmul(Lm[i][k], Um[k][j])
                acc = (acc[0] + t[0], acc[1] + t[1])
            LU[i][j] = acc
    perm = rng.permutation(n)  # row i of L U sits at row perm[i] of A
    A = [[zero] * n for _ in range(n)]
    for i in range(n):
        A[perm[i]] = LU[i]
    # the interchanges partial pivoting makes: at column c, the row holding L U's row c
    cur = [0] * n
    for i in range(n):
        cur[perm[i]] = i
    ipiv = []
    for c in range(n):
        r = cur.index(c, c)
        ipiv.append(r)
        cur[c], cur[r] = cur[r], cur[c]
    packed = [[Lm[i][j] if i > j else Um[i][j] for j in range(n)] for i in range(n)]
    x = [(Fraction(k + 1), Fraction(k + 1)) for k in range(n)]  # x_k = k + k i, k = 1 .. n
    b = []
    for i in range(n):
        acc = zero
        for k in range(n):
            t = _cmul(A[i][k], x[k])
            acc = (acc[0] + t[0], acc[1] + t[1])
        b.append(acc)
    return {"A": A, "packed": packed, "ipiv": np.array(ipiv, np.int32), "x": x, "b": b}


def to_cmat(vals, prec_bits: int):
    """[rows][cols] of (re, im) exact values -> HostCMat."""
    return cmat_from_values([[v[0] for v in row] for row in vals], [[v[1] for v in row] for row in vals], prec_bits)


def column(vals):
    return [[v] for v in vals]


def dominant_matrix(n: int, prec_bits: int, seed, exp_range: int = 2):
    """The factorization workload: random entries (exponents on [-R, R]) plus
    n (1 + i) on the diagonal, each shifted diagonal component rounded once to
    prec_bits (nearest, ties to even) from its exact value."""
    from mpgen import random_cmat
    from oracle.fraction_ref import decode, round_rne
    from tests.mp_util import encode
    A = random_cmat(seed, 0, n, n, prec_bits, exp_range)
    for part in (A.re, A.im):
        for i in range(n):
            s, e, q = round_rne(decode(part, i, i, prec_bits) + n, prec_bits)
            sg, ex, limbs = encode((-q if s else q, e - prec_bits), prec_bits)
            part.sign[i, i] = sg
            part.exp[i, i] = ex
            for l in range(part.L):
                part.mant[l, i, i] = np.uint64(limbs[l])
    return A


def diagonal_pivots(n: int, prec_bits: int, seed):
    """An n x n diagonal matrix of pivots of every kind the reciprocal meets:
    random significands, real and imaginary parts close in exponent, far
    apart (near the width at which the smaller square stops mattering, and
    twice beyond it), one part zero, powers of two, all-ones significands."""
    from mpgen import EXP_ZERO, random_cmat
    A = random_cmat(seed, 0, n, n, prec_bits, 6)
    rng = np.random.default_rng([int(s) for s in np.atleast_1d(seed)] + [99])
    L = A.re.L
    wide = (3 * prec_bits + 7) // 2
    for part in (A.re, A.im):
        off = ~np.eye(n, dtype=bool)
        part.exp[off] = EXP_ZERO
        part.mant[:, off] = 0
        part.sign[off] = 0
    for i in range(n):
        kind = i % 8
        if kind == 1:
            A.im.exp[i, i] = A.re.exp[i, i] + int(rng.choice([-1, 1])) * (wide + int(rng.integers(-2, 3)))
        elif kind == 2:
            A.im.exp[i, i] = A.re.exp[i, i] + int(rng.integers(-3 * prec_bits, 3 * prec_bits + 1))
        elif kind == 3:
            part = A.re if rng.random() < 0.5 else A.im
            part.exp[i, i] = EXP_ZERO
            part.mant[:, i, i] = 0
        elif kind == 4:
            for part in (A.re, A.im):
                part.mant[:, i, i] = 0
                part.mant[L - 1, i, i] = np.uint64(1 << 63)
        elif kind == 5:
            for part in (A.re, A.im):
                M = ((1 << prec_bits) - 1) << (64 * L - prec_bits)
                for l in range(L):
                    part.mant[l, i, i] = np.uint64((M >> (64 * l)) & ((1 << 64) - 1))
        elif kind == 6:  # far beyond that width (the factorization's own products then need ~3p/7 more slices)
            A.im.exp[i, i] = A.re.exp[i, i] + int(rng.choice([-1, 1])) * (3 * prec_bits + int(rng.integers(0, 200)))
    return A
