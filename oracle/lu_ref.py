"""Blocked complex LU with partial pivoting, and the solve with its factors
(Sec. IV-B: the right-looking factorization of width K whose trailing
updates A22 - L21 U12 are matrix products; forward and backward substitution).

TEST INFRASTRUCTURE ONLY: the tests are the only callers.  The paper runs the
factorization in multi-precision arithmetic without fixing its order of
operations or its division; this module writes out the order the library
uses, step by step, with every product and update taken from the oracle's
correctly rounded ``cgemm`` / ``cgemm_acc`` (one rounding per component of
the exact result):

* pivot of column c: the first row r >= c with the largest RNE(|Re| + |Im|)
  (LAPACK's magnitude |Re| + |Im|, rounded once), rows c and r exchanged over
  the whole matrix;
* reciprocal of a pivot y: each component of the exact 1/y rounded once to
  p bits, RNE_p(Re y / |y|^2) and RNE_p(-Im y / |y|^2) (the correctly rounded
  division of MPC arithmetic, Sec. II), written here with exact rationals;
  a zero y gives zero;
* the column below the pivot times the reciprocal; a rank-1 update of the
  rest of the block column; U12 := L11^-1 A12 by rank-1 updates; A22 := A22 -
  L21 U12 in one product;
* solve: interchanges, Y_c := RNE(B_c - L(c, :c) Y(:c)) for c = 1 .. n-1,
  then X_c := RNE(RNE(Y_c - U(c, c+1:) X(c+1:)) * reciprocal of U(c, c)) for c
  = n-1 .. 0.
"""
from __future__ import annotations

import numpy as np

import oracle
from mpgen import EXP_ZERO, HostCMat, HostPart, limbs_for
from fractions import Fraction

from oracle.fraction_ref import decode, round_rne


def _sub(M: HostCMat, r0: int, nr: int, c0: int, nc: int) -> HostCMat:
    """Copy of the nr x nc block at (r0, c0), leading dimension nr."""
    def part(p: HostPart) -> HostPart:
        return HostPart(nr, nc, nr, p.L, p.sign[c0:c0 + nc, r0:r0 + nr].copy(),
                        p.exp[c0:c0 + nc, r0:r0 + nr].copy(), p.mant[:, c0:c0 + nc, r0:r0 + nr].copy())
    return HostCMat(part(M.re), part(M.im))


def _put(M: HostCMat, r0: int, c0: int, S: HostCMat) -> None:
    for d, s in ((M.re, S.re), (M.im, S.im)):
        d.sign[c0:c0 + S.cols, r0:r0 + S.rows] = s.sign[:S.cols, :S.rows]
        d.exp[c0:c0 + S.cols, r0:r0 + S.rows] = s.exp[:S.cols, :S.rows]
        d.mant[:, c0:c0 + S.cols, r0:r0 + S.rows] = s.mant[:, :S.cols, :S.rows]


def _swap_rows(M: HostCMat, a: int, b: int) -> None:
    if a == b:
        return
    for p in (M.re, M.im):
        p.sign[:, [a, b]] = p.sign[:, [b, a]]
        p.exp[:, [a, b]] = p.exp[:, [b, a]]
        p.mant[:, :, [a, b]] = p.mant[:, :, [b, a]]


def _small(v: int, prec_bits: int) -> HostPart:
    """1 x 1 component holding v in {-1, 0, 1}."""
    L = limbs_for(prec_bits)
    mant = np.zeros((L, 1, 1), np.uint64)
    if v:
        mant[L - 1, 0, 0] = np.uint64(1 << 63)
    return HostPart(1, 1, 1, L, np.array([[1 if v < 0 else 0]], np.uint8),
                    np.array([[1 if v else EXP_ZERO]], np.int32), mant)


def _const(vre: int, vim: int, prec_bits: int) -> HostCMat:
    return HostCMat(_small(vre, prec_bits), _small(vim, prec_bits))


def _abs(S: HostCMat) -> HostCMat:
    T = S.copy()
    T.re.sign[...] = 0
    T.im.sign[...] = 0
    return T


def _store(part: HostPart, value: Fraction, prec_bits: int) -> None:
    """Entry (0, 0) of `part` := RNE_p(value) (an exact zero is +0)."""
    sg, e, q = round_rne(value, prec_bits)
    L = part.L
    part.mant[:, 0, 0] = 0
    if q == 0:
        part.sign[0, 0] = 0
        part.exp[0, 0] = EXP_ZERO
        return
    M = q << (64 * L - prec_bits)
    part.sign[0, 0] = sg
    part.exp[0, 0] = e
    for l in range(L):
        part.mant[l, 0, 0] = np.uint64((M >> (64 * l)) & ((1 << 64) - 1))


def reciprocal(y: HostCMat, prec_bits: int) -> HostCMat:
    """The reciprocal of a 1 x 1 y, correctly rounded in each component:
    RNE_p(Re y / |y|^2) + i RNE_p(-Im y / |y|^2) from exact rationals; zero
    for y = 0."""
    yr = decode(y.re, 0, 0, prec_bits)
    yi = decode(y.im, 0, 0, prec_bits)
    x = _const(0, 0, prec_bits)
    d = yr * yr + yi * yi
    if d == 0:
        return x
    _store(x.re, yr / d, prec_bits)
    _store(x.im, -yi / d, prec_bits)
    return x


def _first_max(K: HostCMat, prec_bits: int) -> int:
    best, bv = 0, None
    for i in range(K.rows):
        v = decode(K.re, i, 0, prec_bits)
        if bv is None or v > bv:
            best, bv = i, v
    return best


def getrf(A: HostCMat, nb: int, prec_bits: int):
    """Returns (LU packed in one matrix, ipiv (0-based), info)."""
    n = A.rows
    assert A.cols == n
    M = _sub(A, 0, n, 0, n)
    ipiv = np.zeros(n, np.int32)
    info = 0
    omi = _const(1, -1, prec_bits)
    nb = nb or 64
    p = prec_bits
    for j in range(0, n, nb):
        jb = min(nb, n - j)
        for c in range(j, j + jb):
            mr = n - c
            K = oracle.cgemm(_abs(_sub(M, c, mr, c, 1)), omi, p)
            r = c + _first_max(K, p)
            ipiv[c] = r
            if K.re.exp[0, r - c] == EXP_ZERO and info == 0:
                info = c + 1
            _swap_rows(M, c, r)
            R = reciprocal(_sub(M, c, 1, c, 1), p)
            if mr > 1:
                _put(M, c + 1, c, oracle.cgemm(_sub(M, c + 1, mr - 1, c, 1), R, p))
                w = j + jb - c - 1
                if w > 0:
                    _put(M, c + 1, c + 1, oracle.cgemm_acc(_sub(M, c + 1, mr - 1, c, 1), _sub(M, c, 1, c + 1, w),
                                                           _sub(M, c + 1, mr - 1, c + 1, w), p, sign=-1))
        nr = n - j - jb
        if nr > 0:
            for c in range(j, j + jb - 1):
                h = j + jb - c - 1
                _put(M, c + 1, j + jb, oracle.cgemm_acc(_sub(M, c + 1, h, c, 1), _sub(M, c, 1, j + jb, nr),
                                                        _sub(M, c + 1, h, j + jb, nr), p, sign=-1))
            _put(M, j + jb, j + jb, oracle.cgemm_acc(_sub(M, j + jb, nr, j, jb), _sub(M, j, jb, j + jb, nr),
                                                     _sub(M, j + jb, nr, j + jb, nr), p, sign=-1))
    return M, ipiv, info


def getrs(LU: HostCMat, ipiv, B: HostCMat, prec_bits: int) -> HostCMat:
    """X with A X = B from getrf's factors."""
    n, nrhs = LU.rows, B.cols
    X = _sub(B, 0, n, 0, nrhs)
    p = prec_bits
    for c in range(n):
        _swap_rows(X, c, int(ipiv[c]))
    for c in range(1, n):
        _put(X, c, 0, oracle.cgemm_acc(_sub(LU, c, 1, 0, c), _sub(X, 0, c, 0, nrhs), _sub(X, c, 1, 0, nrhs), p,
                                       sign=-1))
    for c in range(n - 1, -1, -1):
        if c + 1 < n:
            _put(X, c, 0, oracle.cgemm_acc(_sub(LU, c, 1, c + 1, n - c - 1), _sub(X, c + 1, n - c - 1, 0, nrhs),
                                           _sub(X, c, 1, 0, nrhs), p, sign=-1))
        R = reciprocal(_sub(LU, c, 1, c, 1), p)
        _put(X, c, 0, oracle.cgemm(R, _sub(X, c, 1, 0, nrhs), p))
    return X
