"""Device path vs the CPU oracle, bit for bit (exact scheme) on seeded inputs.

Every call goes through the C-ABI (libmpcgemm.so) via the thin binding.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, random_cmat, workload_inputs
from tests.gpu_util import mismatches, run_device

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT, TRUNC = 0, 1
I8, F64 = 0, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check_exact(A, B, p, mode, slice_type=I8, **kw):
    m, n = A.rows, B.cols
    _say(f"case m={m} n={n} k={A.cols} p={p} mode={mode} slice={slice_type} {kw}")
    C, info = run_device(A, B, p, mode, EXACT, slice_type, **kw)
    R = oracle.cgemm(A, B, p)
    bad, first = mismatches(C, R, m, n)
    assert bad == 0, f"{bad} mismatching components, first {first}, info {info}"
    return info


@pytest.mark.parametrize("mode", [M4, M3])
@pytest.mark.parametrize("slice_type", [I8, F64])
def test_small_square_exact(mode, slice_type):
    # 64 x 64 x 64 at 256 bits, exponents in [-4, 4]
    m, n, k, p, A, B = workload_inputs("cgemm64_p256")
    info = _check_exact(A, B, p, mode, slice_type)
    assert info["nprod"] == (3 if mode == M3 else 4)


@pytest.mark.parametrize("mode", [M4, M3])
@pytest.mark.parametrize("slice_type", [I8, F64])
@pytest.mark.parametrize("shape", [(37, 45, 71), (1, 1, 1), (16, 48, 130), (50, 3, 200)])
def test_ragged_exact(mode, slice_type, shape):
    m, n, k = shape
    p = 130
    A = random_cmat(11, 0, m, k, p, 10, zero_frac=0.15)
    B = random_cmat(11, 1, k, n, p, 10, zero_frac=0.15)
    _check_exact(A, B, p, mode, slice_type)


@pytest.mark.parametrize("block", [8, 12, 16, 20])
@pytest.mark.parametrize("ksplit", [1, 2, 3])
def test_tiling_independent(block, ksplit):
    """Band width and contraction chunks never change the bits."""
    m, n, k, p = 40, 36, 300, 200
    A = random_cmat(5, 0, m, k, p, 6)
    B = random_cmat(5, 1, k, n, p, 6)
    _check_exact(A, B, p, M3, I8, block_override=block, ksplit_override=ksplit)
    _check_exact(A, B, p, M4, I8, block_override=block, ksplit_override=ksplit)


_APART_REF = {}


def _apart_ref():
    """512^3 at 512 bits: the inputs, sampled oracle entries (corners
    included) and the fused 3M kernel's whole result (band 20)."""
    if "ref" not in _APART_REF:
        m, n, k, p, A, B = workload_inputs("cgemm512_p512")
        rng = np.random.default_rng(7)
        rows = np.concatenate([rng.integers(0, m, 300), [0, m - 1, 0, m - 1]])
        cols = np.concatenate([rng.integers(0, n, 300), [0, 0, n - 1, n - 1]])
        ent = oracle.cgemm_entries(A, B, rows, cols, p)
        C20, info = run_device(A, B, p, M3, EXACT, I8, block_override=20)
        assert info["apart"] == 0, info
        _APART_REF["ref"] = (m, n, k, p, A, B, rows, cols, ent, C20)
    return _APART_REF["ref"]


@pytest.mark.parametrize("mode,block,apart", [(M3, 0, 1), (M3, 8, 1), (M3, 12, 1), (M3, 16, 1), (M4, 0, 1),
                                              (M4, 12, 1)])
def test_products_apart(mode, block, apart):
    """A product whose contraction is long enough for it (k S >= 2^14 (ks +
    1): here 512 x 67 in one contraction chunk) runs each real product on
    workgroups of its own with bands of at most 16 diagonals: a digit stream
    per product (3M: T3's holding Im digits only; 4M: each product's one
    component), added up by the rounding.  Every form gives the oracle's bits
    on the sampled entries and the fused 3M kernel's (band 20) everywhere."""
    m, n, k, p, A, B, rows, cols, (s, e, mm), C20 = _apart_ref()
    _say(f"case m={m} n={n} k={k} p={p} mode={mode} block={block}")
    C, info = run_device(A, B, p, mode, EXACT, I8, block_override=block)
    assert info["apart"] == apart, info
    if apart:
        assert info["block"] <= 16 and info["ksplit"] == 1, info
    bad, first = mismatches(C, C20, m, n)
    assert bad == 0, f"{bad} components differ from the fused kernel's, first {first}, info {info}"
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((C.re, C.im)):
            assert part.exp[j, i] == e[t, comp], (i, j, comp)
            if e[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == s[t, comp]
                assert np.array_equal(part.mant[:, j, i], mm[t, comp])


@pytest.mark.parametrize("m,k,apart", [(1024, 128, 0), (256, 256, 1)])
def test_short_contraction(m, k, apart):
    """At 256 bits k S stays below 2^14 (ks + 1): a product whose products
    together fill the chip (1024 tile groups x 1 chunk, a rank-128 update)
    keeps them together; one of fewer work items (64 tile groups x 4 chunks)
    runs them apart.  Sampled oracle entries, corners included."""
    n, p = m, 256
    A = random_cmat(22, 0, m, k, p, 4)
    B = random_cmat(22, 1, k, n, p, 4)
    _say(f"case m={m} n={n} k={k} p={p}")
    C, info = run_device(A, B, p, M3, EXACT, I8)
    assert info["apart"] == apart, info
    rng = np.random.default_rng(3)
    rows = np.concatenate([rng.integers(0, m, 400), [0, m - 1, 0, m - 1]])
    cols = np.concatenate([rng.integers(0, n, 400), [0, 0, n - 1, n - 1]])
    s, e, mm = oracle.cgemm_entries(A, B, rows, cols, p)
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((C.re, C.im)):
            assert part.exp[j, i] == e[t, comp], (i, j, comp)
            if e[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == s[t, comp]
                assert np.array_equal(part.mant[:, j, i], mm[t, comp])


@pytest.mark.parametrize("mode", [M3, M4])
@pytest.mark.parametrize("shape", [(1, 1, 320), (3, 5, 448), (17, 9, 500)])
def test_band_groups_many_chunks(mode, shape):
    """A tiny output with a long contraction: 5 to 8 contraction chunks, its
    bands in groups on workgroups of their own, so the rounding merges more
    than four streams per band group and adds every group's carry at the next
    group's first digit."""
    m, n, k = shape
    p = 200
    A = random_cmat([12, m, n, k], 0, m, k, p, 7, zero_frac=0.1)
    B = random_cmat([12, m, n, k], 1, k, n, p, 7, zero_frac=0.1)
    info = _check_exact(A, B, p, mode, I8)
    assert info["ksplit"] >= 5, info


@pytest.mark.parametrize("p", [2, 3, 53, 64, 65, 127, 512, 1024])
def test_precisions(p):
    A = random_cmat(p, 0, 20, 33, p, 5)
    B = random_cmat(p, 1, 33, 18, p, 5)
    _check_exact(A, B, p, M3)
    _check_exact(A, B, p, M4)


@pytest.mark.parametrize("p", [2047, 3000, 4096])
def test_wide_precisions(p):
    """Up to the largest supported precision (4096 bits, 64 limbs): the
    rounding kernel's binary window of |X| then spans 65 words per thread."""
    A = random_cmat(p, 0, 9, 14, p, 6, zero_frac=0.05)
    B = random_cmat(p, 1, 14, 11, p, 6, zero_frac=0.05)
    _check_exact(A, B, p, M3)
    _check_exact(A, B, p, M4)


def test_wide_exponent_spread():
    p = 96
    A = random_cmat(21, 0, 24, 40, p, 70)
    B = random_cmat(21, 1, 40, 24, p, 70)
    _check_exact(A, B, p, M3)
    _check_exact(A, B, p, M4, F64)


def test_all_zero_and_k_zero():
    p = 64
    A = random_cmat(3, 0, 8, 8, p, 2, zero_frac=1.0)
    B = random_cmat(3, 1, 8, 8, p, 2)
    C, _ = run_device(A, B, p, M3, EXACT)
    assert (C.re.exp[:8, :8] == EXP_ZERO).all() and (C.im.exp[:8, :8] == EXP_ZERO).all()


def test_cancellation_to_zero():
    """Terms that cancel exactly: full cancellation gives +0, partial cancellation stays exact."""
    p = 64
    for k in (2, 10):
        A = random_cmat(8, 0, 6, k, p, 3)
        B = random_cmat(8, 1, k, 6, p, 3)
        # column 1 of A is minus column 0, row 1 of B equals row 0: those terms cancel
        for part in (A.re, A.im):
            part.exp[1] = part.exp[0]
            part.mant[:, 1] = part.mant[:, 0]
            part.sign[1] = part.sign[0] ^ 1
        for part in (B.re, B.im):
            part.exp[:, 1] = part.exp[:, 0]
            part.mant[:, :, 1] = part.mant[:, :, 0]
            part.sign[:, 1] = part.sign[:, 0]
        _check_exact(A, B, p, M3)
        _check_exact(A, B, p, M4)
        if k == 2:
            C, _ = run_device(A, B, p, M3, EXACT)
            assert (C.re.exp[:6, :6] == EXP_ZERO).all() and (C.im.exp[:6, :6] == EXP_ZERO).all()


def test_config_512_p512_sampled():
    """512 x 512 x 512 at 512 bits: every output checked on a sample, all 4 forms."""
    m, n, k, p, A, B = workload_inputs("cgemm512_p512")
    rng = np.random.default_rng(2)
    rows = np.concatenate([rng.integers(0, m, 600), [0, m - 1, 0, m - 1]])
    cols = np.concatenate([rng.integers(0, n, 600), [0, 0, n - 1, n - 1]])
    s, e, mm = oracle.cgemm_entries(A, B, rows, cols, p)
    for mode, st in [(M3, I8), (M4, I8), (M4, F64)]:
        _say(f"config512 mode={mode} slice={st}")
        C, info = run_device(A, B, p, mode, EXACT, st)
        for t, (i, j) in enumerate(zip(rows, cols)):
            for comp, part in enumerate((C.re, C.im)):
                assert part.exp[j, i] == e[t, comp], (mode, st, i, j, comp)
                if e[t, comp] != EXP_ZERO:
                    assert part.sign[j, i] == s[t, comp]
                    assert np.array_equal(part.mant[:, j, i], mm[t, comp])


@pytest.mark.parametrize("p", [64, 128, 192])
def test_rounding_bit_below_limb_zero(p):
    """p = 64 L puts the rounding bit one below the lowest significand limb; on
    every 112th component or so that bit opens a new 16-digit chunk.  Whole
    matrices, bit for bit, so many such components are checked."""
    m, n, k = 160, 144, 40
    A = random_cmat(90 + p, 0, m, k, p, 12)
    B = random_cmat(90 + p, 1, k, n, p, 12)
    _check_exact(A, B, p, M3)
    _check_exact(A, B, p, M4)


@pytest.mark.parametrize("mode", [M4, M3])
@pytest.mark.parametrize("shape,p", [((40, 36, 1), 256), ((17, 70, 2), 130), ((100, 3, 5), 512), ((33, 33, 8), 64),
                                     ((20, 18, 9), 200), ((16, 16, 1), 4096), ((1, 40, 3), 1000)])
def test_short_contraction(mode, shape, p):
    """Contractions of 1 to 9 (one 64-wide block, mostly padding), at 64 to
    4096 bits: few work items, so each band runs on a workgroup of its own
    and the rounding adds the bands' streams.  Exact bits."""
    m, n, k = shape
    A = random_cmat([81, m, n, k], 0, m, k, p, 9, zero_frac=0.1)
    B = random_cmat([81, m, n, k], 1, k, n, p, 9, zero_frac=0.1)
    _check_exact(A, B, p, mode)
