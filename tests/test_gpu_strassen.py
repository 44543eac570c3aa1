"""One level of Strassen's recursion over the slice products (the strassen
option): the same bits as the oracle's plain product, element by element, on
ragged and structured inputs (rows folded together with far-apart
exponents, operand sums that cancel to zero, zero quadrants, several
contraction chunks), the plain product where the recursion does not apply,
and sampled entries of the 2048 x 2048 x 2048 workload at 1024 bits."""
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


def _check(A, B, p, mode, expect_strassen=1, **kw):
    m, n = A.rows, B.cols
    _say(f"strassen m={m} n={n} k={A.cols} p={p} mode={mode} {kw}")
    C, info = run_device(A, B, p, mode, EXACT, I8, strassen=1, **kw)
    assert info["strassen"] == expect_strassen, info
    R = oracle.cgemm(A, B, p)
    bad, first = mismatches(C, R, m, n)
    assert bad == 0, f"{bad} mismatching components, first {first}, info {info}"
    return info


@pytest.mark.parametrize("mode", [M4, M3])
@pytest.mark.parametrize("shape,p,R,zf", [
    ((32, 32, 64), 256, 4, 0.0),
    ((34, 66, 130), 130, 10, 0.15),   # half sizes 17 x 33 x 65: ragged tiles everywhere
    ((2, 2, 2), 64, 3, 0.0),
    ((100, 36, 200), 200, 6, 0.05),
    ((64, 64, 64), 1024, 3, 0.0),
    ((48, 80, 40), 53, 20, 0.3),
])
def test_parity(mode, shape, p, R, zf):
    """Half-size products this small run their real products apart (3M: T3's
    streams without Re digits; 4M: each product's one component), so the
    quadrant merges take separate Re and Im source lists."""
    m, n, k = shape
    A = random_cmat([61, m, n, k], 0, m, k, p, R, zero_frac=zf)
    B = random_cmat([61, m, n, k], 1, k, n, p, R, zero_frac=zf)
    info = _check(A, B, p, mode)
    assert info["apart"] == 1, info


@pytest.mark.parametrize("mode", [M4, M3])
def test_folded_rows_far_apart(mode):
    """Rows r and r + m/2 of A (columns c and c + n/2 of B) share a scale in
    every operand combination; their exponents 80 (70) apart widen the
    folded spread, and the slices still hold every bit."""
    m, n, k, p = 40, 48, 96, 192
    A = random_cmat(62, 0, m, k, p, 5)
    B = random_cmat(62, 1, k, n, p, 5)
    for part in (A.re, A.im):
        scale_exponents(part, rows=list(range(m // 2)), shift=40)
        scale_exponents(part, rows=list(range(m // 2, m)), shift=-40)
    for part in (B.re, B.im):
        scale_exponents(part, cols=list(range(n // 2, n)), shift=-70)
    info = _check(A, B, p, mode)
    assert info["S_A"] * info["w"] >= p + 80


def _copy_block(dst, src, r0, c0, r1, c1, h, w, negate=False):
    """dst[r1:r1+h, c1:c1+w] := (-)src[r0:r0+h, c0:c0+w] (both parts)."""
    for name in ("re", "im"):
        d, s = getattr(dst, name), getattr(src, name)
        d.exp[c1:c1 + w, r1:r1 + h] = s.exp[c0:c0 + w, r0:r0 + h]
        d.mant[:, c1:c1 + w, r1:r1 + h] = s.mant[:, c0:c0 + w, r0:r0 + h]
        sg = s.sign[c0:c0 + w, r0:r0 + h].copy()
        if negate:
            sg = np.where(s.exp[c0:c0 + w, r0:r0 + h] == EXP_ZERO, 0, 1 - sg).astype(np.uint8)
        d.sign[c1:c1 + w, r1:r1 + h] = sg


def _zero_block(dst, r, c, h, w):
    for name in ("re", "im"):
        d = getattr(dst, name)
        d.exp[c:c + w, r:r + h] = EXP_ZERO
        d.sign[c:c + w, r:r + h] = 0
        d.mant[:, c:c + w, r:r + h] = 0


@pytest.mark.parametrize("mode", [M4, M3])
def test_cancelling_sums_and_zero_quadrants(mode):
    """A21 = A11 (M6's left operand is exactly zero), B22 = -B11 (M1's right
    operand is exactly zero), A12 = 0 and B21 = 0: products of exact zeros
    and quadrants of C that are sums of zero and nonzero products."""
    m, n, k, p = 32, 64, 128, 256
    hm, hn, hk = m // 2, n // 2, k // 2
    A = random_cmat(63, 0, m, k, p, 6)
    B = random_cmat(63, 1, k, n, p, 6)
    _copy_block(A, A, 0, 0, hm, 0, hm, hk)
    _copy_block(B, B, 0, 0, hk, hn, hk, hn, negate=True)
    _zero_block(A, 0, hk, hm, hk)
    _zero_block(B, hk, 0, hk, hn)
    _check(A, B, p, mode)


@pytest.mark.parametrize("ksplit,expect", [(2, 1), (3, 1), (4, 1), (5, 1), (7, 1), (14, 0)])
def test_contraction_chunks(ksplit, expect):
    """The half-size products in 2 to 7 contraction chunks merge every
    stream into the quadrants (up to 4 chunks with each 3M real product on
    workgroups of its own, a stream per chunk and product: at most 48 per
    quadrant; from 5 chunks the products together); 14 would exceed the
    merge's 48 streams and the plain product runs."""
    m, n, k, p = 36, 40, 1792, 160  # 14 blocks of 64 in the half contraction
    A = random_cmat(64, 0, m, k, p, 8)
    B = random_cmat(64, 1, k, n, p, 8)
    info = _check(A, B, p, M3, expect, ksplit_override=ksplit)
    assert info["ksplit"] == ksplit


@pytest.mark.parametrize("shape", [(33, 32, 32), (32, 31, 32), (32, 32, 63), (1, 2, 2)])
def test_odd_sizes_run_plain(shape):
    m, n, k = shape
    p = 128
    A = random_cmat(65, 0, m, k, p, 4)
    B = random_cmat(65, 1, k, n, p, 4)
    _check(A, B, p, M3, 0)


def test_zero_half_of_every_folded_pair():
    """B's first n/2 columns all zero: every folded column pair takes its
    scale from the nonzero column alone, and M2, M4 and M6 multiply by
    operands whose B11 part is zero."""
    m, n, k, p = 16, 16, 32, 128
    A = random_cmat(66, 0, m, k, p, 4)
    B = random_cmat(66, 1, k, n, p, 4)
    _zero_block(B, 0, 0, k, n // 2)
    _check(A, B, p, M4)


def test_agrees_with_plain_512():
    """512 x 512 x 512 at 256 bits: the recursion's bits equal the plain
    product's everywhere, and sampled entries equal the oracle's."""
    m = n = k = 512
    p = 256
    A = random_cmat(67, 0, m, k, p, 8)
    B = random_cmat(67, 1, k, n, p, 8)
    _say("512^3 p=256: plain and recursive 3M")
    C0, _ = run_device(A, B, p, M3, EXACT, I8)
    C1, info = run_device(A, B, p, M3, EXACT, I8, strassen=1)
    assert info["strassen"] == 1
    bad, first = mismatches(C1, C0, m, n)
    assert bad == 0, (bad, first)
    rng = np.random.default_rng(67)
    ri, ci = rng.integers(0, m, 64), rng.integers(0, n, 64)
    s, e, mm = oracle.cgemm_entries(A, B, ri, ci, p)
    for t, (i, j) in enumerate(zip(ri, ci)):
        for comp, part in enumerate((C1.re, C1.im)):
            assert part.exp[j, i] == e[t, comp]
            if e[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == s[t, comp] and np.array_equal(part.mant[:, j, i], mm[t, comp])


@pytest.mark.parametrize("mode", [M3, M4])
def test_config_2048_p1024_sampled(mode):
    """The benchmark's 2048 x 2048 x 2048 workload at 1024 bits with the
    recursion, on sampled entries (two full rows and columns at a stride)."""
    from tests.test_gpu_scale import _check_sampled, _sample
    m, n, k, p, A, B = workload_inputs("cgemm2048_p1024")
    ri, ci = _sample(m, n, 8, 300, (0, m // 2, m - 1), (n // 2 - 1,))
    _say(f"cgemm2048_p1024 strassen mode={mode}: oracle on {ri.size} entries")
    s, e, mm = oracle.cgemm_entries(A, B, ri, ci, p)
    _say("  device")
    C, info = run_device(A, B, p, mode, EXACT, I8, strassen=1)
    _say(f"  S_A={info['S_A']} S_B={info['S_B']} ksplit={info['ksplit']} block={info['block']}")
    assert info["strassen"] == 1
    _check_sampled(C, ri, ci, s, e, mm, f"strassen {mode}")


def test_falls_back_when_the_workspace_is_short():
    """With a caller workspace sized for the plain product (the workspace
    query at the largest spread the inputs can have), the recursion's seven
    plan layouts do not fit: the plain product runs in it, with no error and
    the oracle's bits."""
    import torch
    import paper_2307_06072_amd as mp
    m = n = k = 256
    p, R = 256, 6
    A = random_cmat(68, 0, m, k, p, R)
    B = random_cmat(68, 1, k, n, p, R)
    wsz = mp.mpcg_workspace_size(m, n, k, p, M3, EXACT, None, 2 * R)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    mp.mpcg_set_workspace(ws.data_ptr(), wsz)
    try:
        _say("short workspace, strassen=1")
        C, info = run_device(A, B, p, M3, EXACT, I8, strassen=1)
        assert info["strassen"] == 0, info
        bad, first = mismatches(C, oracle.cgemm(A, B, p), m, n)
        assert bad == 0, (bad, first)
    finally:
        mp.mpcg_set_workspace(None, 0)
