"""Separate scales for the Re and Im parts (the part_scales option, 4M):
bit parity with the oracle where imaginary parts sit far below or above the
real ones, with gaps that differ per row and column and are not multiples of
the digit width, zero parts, a real component that cancels exactly between
two products at scales 192 bits apart, several contraction chunks; fewer
slice pairs than one scale per row; the one-scale product where the option
does not apply; sampled entries of the 2048 x 2048 x 2048 workload at 1024
bits with every imaginary part 2^200 below the real parts."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, random_cmat, scale_exponents, workload_inputs
from tests.gpu_util import mismatches, run_device

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT = 0
I8 = 0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(A, B, p, expect=1, mode=M4, **kw):
    m, n = A.rows, B.cols
    _say(f"parts m={m} n={n} k={A.cols} p={p} mode={mode} {kw}")
    C, info = run_device(A, B, p, mode, EXACT, I8, part_scales=1, **kw)
    assert info["part_scales"] == expect, info
    R = oracle.cgemm(A, B, p)
    bad, first = mismatches(C, R, m, n)
    assert bad == 0, f"{bad} mismatching components, first {first}, info {info}"
    return C, info


def _shift_rows(part, shifts):
    for r, sh in enumerate(shifts):
        scale_exponents(part, rows=[r], shift=int(sh))


def _shift_cols(part, shifts):
    for c, sh in enumerate(shifts):
        scale_exponents(part, cols=[c], shift=int(sh))


@pytest.mark.parametrize("shape,p", [((40, 36, 70), 192), ((17, 33, 65), 130), ((1, 1, 1), 64),
                                     ((64, 48, 256), 512)])
def test_imaginary_parts_far_below(shape, p):
    m, n, k = shape
    zf = 0.05 if k > 1 else 0.0
    A = random_cmat([71, m, n, k], 0, m, k, p, 6, zero_frac=zf)
    B = random_cmat([71, m, n, k], 1, k, n, p, 6, zero_frac=zf)
    scale_exponents(A.im, rows=list(range(m)), shift=-200)
    scale_exponents(B.im, rows=list(range(k)), shift=-200)
    _, info0 = run_device(A, B, p, M4, EXACT, I8)
    _, info1 = _check(A, B, p)
    assert info1["pairs"] < info0["pairs"], (info0, info1)


def test_gaps_per_row_and_column():
    """Im above Re in some rows of A, below in others, by amounts that are not
    multiples of 8; B's columns likewise: the digit shifts between a
    component's two products take both signs."""
    m, n, k, p = 48, 40, 96, 256
    rng = np.random.default_rng(72)
    A = random_cmat(72, 0, m, k, p, 5)
    B = random_cmat(72, 1, k, n, p, 5)
    _shift_rows(A.im, rng.integers(-170, 171, m))
    _shift_cols(B.im, rng.integers(-130, 131, n))
    _check(A, B, p)


def test_zero_parts():
    """Rows of A with no imaginary part, rows with no real part, columns of B
    likewise, and an all-zero row and column."""
    m, n, k, p = 36, 28, 64, 160
    A = random_cmat(73, 0, m, k, p, 4)
    B = random_cmat(73, 1, k, n, p, 4)
    scale_exponents(A.im, rows=list(range(m)), shift=-120)
    scale_exponents(B.im, rows=list(range(k)), shift=90)
    for part, rows in ((A.im, range(0, 8)), (A.re, range(8, 14)), (A.re, [20]), (A.im, [20])):
        for r in rows:
            part.exp[:, r] = EXP_ZERO
    for part, cols in ((B.im, range(0, 5)), (B.re, range(5, 9)), (B.re, [11]), (B.im, [11])):
        for c in cols:
            part.exp[c, :] = EXP_ZERO
    _check(A, B, p)


def test_exact_cancellation_across_scales():
    """Im A = Re A 2^-96 and Im B = Re B 2^96: Re C = Re A Re B - Im A Im B is
    exactly zero although its two products sit 192 bits apart; Im C is the
    sum of two products at the same scale."""
    m, n, k, p = 32, 32, 48, 256
    A = random_cmat(74, 0, m, k, p, 6)
    B = random_cmat(74, 1, k, n, p, 6)
    for X, sh in ((A, -96), (B, 96)):
        X.im.sign[...] = X.re.sign
        X.im.mant[...] = X.re.mant
        X.im.exp[...] = np.where(X.re.exp == EXP_ZERO, EXP_ZERO, X.re.exp + np.int32(sh))
    C, _ = _check(A, B, p)
    assert np.all(C.re.exp[:n, :m] == EXP_ZERO)


@pytest.mark.parametrize("ksplit", [2, 3])
def test_contraction_chunks(ksplit):
    m, n, k, p = 36, 40, 900, 192
    A = random_cmat(75, 0, m, k, p, 8)
    B = random_cmat(75, 1, k, n, p, 8)
    scale_exponents(A.im, rows=list(range(m)), shift=-150)
    scale_exponents(B.im, rows=list(range(k)), shift=-60)
    _, info = _check(A, B, p, ksplit_override=ksplit)
    assert info["ksplit"] == ksplit


def test_one_scale_where_it_needs_no_more_pairs():
    """Re and Im of similar magnitude: separate scales would not save a slice
    pair, so the one-scale product runs; and a 3M request keeps one scale."""
    m, n, k, p = 40, 40, 64, 256
    A = random_cmat(76, 0, m, k, p, 6)
    B = random_cmat(76, 1, k, n, p, 6)
    _check(A, B, p, expect=0)
    scale_exponents(A.im, rows=list(range(m)), shift=-200)
    _check(A, B, p, expect=0, mode=M3)


def test_config_2048_p1024_im200_sampled():
    """2048 x 2048 x 2048 at 1024 bits, every imaginary part 2^200 below the
    real parts: sampled entries against the oracle."""
    from tests.test_gpu_scale import _check_sampled, _sample
    m, n, k, p, A, B = workload_inputs("cgemm2048_p1024_im200")
    ri, ci = _sample(m, n, 9, 300, (0, m - 1), (n - 1,))
    _say(f"cgemm2048_p1024_im200: oracle on {ri.size} entries")
    s, e, mm = oracle.cgemm_entries(A, B, ri, ci, p)
    _say("  device, separate part scales")
    C, info = run_device(A, B, p, M4, EXACT, I8, part_scales=1)
    _say(f"  S_A={info['S_A']} S_B={info['S_B']} pairs={info['pairs']} ksplit={info['ksplit']}")
    assert info["part_scales"] == 1 and info["S_A"] < 150
    _check_sampled(C, ri, ci, s, e, mm, "part scales")
