"""The accumulating product C := C + sign * A B (mp_cgemm_acc), in place on
the device, against the oracle's once-rounded exact sum, bit for bit in the
exact scheme.  The addend's exponents are shifted row by row and column by
column so that one product covers every regime: the addend far below the
product (a signed sticky bit), overlapping it, far above it (the product only
breaks ties), and the addend equal to the rounded product (deep cancellation)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, HostCMat, empty_cmat, random_cmat, scale_exponents
from tests.gpu_util import device_result_to_host, mismatches
from tests.test_gpu_truncated import _absmax_terms

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT, TRUNC = 0, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _regime_addend(seed, m, n, p, R, base_shift):
    """A random addend whose row r is shifted by one of a cycle of offsets
    around the product's scale, and whose odd columns move by a further +-3."""
    C = random_cmat(seed, 2, m, n, p, R, zero_frac=0.1)
    offs = [-4 * p - 90, -p - 5, -p - 1, -p, -40, -3, 0, 0, 1, 3, 40, p, p + 1, p + 5, 4 * p + 90]
    for part in (C.re, C.im):
        for r in range(m):
            scale_exponents(part, rows=[r], shift=base_shift + offs[r % len(offs)])
        scale_exponents(part, cols=list(range(1, n, 2)), shift=3 if seed % 2 else -3)
    return C


def _flip_last_bit(C: HostCMat, p: int, every: int = 2):
    """C +- 1 ulp on every `every`-th entry (the last significand bit flipped)."""
    D = C.copy()
    L = (p + 63) // 64
    bit = np.uint64(1) << np.uint64(64 * L - p)
    for part in (D.re, D.im):
        nz = part.exp != EXP_ZERO
        sel = np.zeros_like(nz)
        sel.reshape(-1)[::every] = True
        sel &= nz
        part.mant[0][sel] ^= bit
    return D


def _run_acc(A, B, Cin, p, sign, mode=M3, scheme=EXACT, **kw):
    import torch
    import paper_2307_06072_amd as mp
    m, k, n = A.rows, A.cols, B.cols
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.to_device(Cin)
    mp.mpcg_set_stream()
    info = mp.mp_cgemm_acc(m, n, k, dA, A.ld, dB, B.ld, dC, dC.ld, p, sign, mode, scheme, **kw)
    torch.cuda.synchronize()
    st = mp.mpcg_stream_status()
    assert st == 0, f"device status {st}: {mp.mpcg_last_error()}"
    return device_result_to_host(dC, p), info


def _check(A, B, Cin, p, sign, mode=M3, **kw):
    m, n = A.rows, B.cols
    _say(f"acc m={m} n={n} k={A.cols} p={p} sign={sign} mode={mode} {kw}")
    got, info = _run_acc(A, B, Cin, p, sign, mode, **kw)
    ref = oracle.cgemm_acc(A, B, Cin, p, sign)
    bad, first = mismatches(got, ref, m, n)
    assert bad == 0, (bad, first, info)
    return info


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("mode", [M3, M4])
@pytest.mark.parametrize("p", [64, 130, 256])
def test_acc_regimes(p, mode, sign):
    m, n, k = 45, 37, 71
    R = 10
    A = random_cmat(200 + p, 0, m, k, p, R, zero_frac=0.05)
    B = random_cmat(200 + p, 1, k, n, p, R, zero_frac=0.05)
    Cin = _regime_addend(300 + p + mode, m, n, p, R, base_shift=R)
    _check(A, B, Cin, p, sign, mode)


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("mode", [M3, M4])
def test_acc_window_limits(mode, sign):
    """Exact two-bit products X_i = 2^100 + 2^-e_i (A row i = [1, 2^-e_i],
    B = [2^100, 1]^T, imaginary parts zero) against addends that step across
    the limits of the one-pass accumulating form: C's leading bit moves from
    145 bits below X's to above it (X reaching more than 64 bits above C is
    left to the general case), and C = -2^100 with the small term moving down
    until the cancelled sum's rounding bit falls below the window."""
    from fractions import Fraction
    from tests.mp_util import cmat_from_values
    p = 128
    cases = []
    for sh in range(-145, 6):
        c = Fraction(2) ** (100 + sh) * (1 + Fraction(1, 128))
        cases.append((50, c if sh % 2 else -c))
    for e in range(0, 90, 3):
        cases.append((e, -Fraction(2) ** 100))
    m = len(cases)
    A = cmat_from_values([[1, Fraction(1, 2 ** e)] for e, _ in cases], [[0, 0] for _ in cases], p)
    B = cmat_from_values([[2 ** 100], [1]], [[0], [0]], p)
    Cin = cmat_from_values([[c] for _, c in cases], [[0] for _ in cases], p)
    assert m == A.rows
    _check(A, B, Cin, p, sign, mode)


@pytest.mark.parametrize("p", [64, 200, 1024])
def test_acc_cancellation(p):
    """Cin = RNE(AB): C - AB is the rounding error of each entry, far below both
    operands; with the last bit flipped the difference is an ulp away."""
    m, n, k = 33, 19, 40
    A = random_cmat(400 + p, 0, m, k, p, 6)
    B = random_cmat(400 + p, 1, k, n, p, 6)
    Rn = oracle.cgemm(A, B, p)
    _check(A, B, Rn, p, -1)
    _check(A, B, _flip_last_bit(Rn, p), p, -1)
    neg = HostCMat(Rn.re.copy(), Rn.im.copy())
    for part in (neg.re, neg.im):
        part.sign[:] ^= (part.exp != EXP_ZERO).astype(np.uint8)
    _check(A, B, neg, p, 1)


@pytest.mark.parametrize("block", [8, 16, 20])
@pytest.mark.parametrize("ksplit", [1, 3])
def test_acc_tiling_independent(block, ksplit):
    p, m, n, k = 190, 40, 36, 300
    A = random_cmat(51, 0, m, k, p, 8)
    B = random_cmat(51, 1, k, n, p, 8)
    Cin = _regime_addend(52, m, n, p, 8, base_shift=8)
    info = _check(A, B, Cin, p, -1, M3, block_override=block, ksplit_override=ksplit)
    assert info["block"] == block


def test_acc_zero_cases():
    import torch
    import paper_2307_06072_amd as mp
    p, m, n, k = 100, 20, 17, 30
    A = random_cmat(61, 0, m, k, p, 6)
    B = random_cmat(61, 1, k, n, p, 6)
    # a zero addend: the plain product, negated for sign = -1
    for sign in (1, -1):
        got, _ = _run_acc(A, B, empty_cmat(m, n, p), p, sign)
        assert mismatches(got, oracle.cgemm_acc(A, B, empty_cmat(m, n, p), p, sign), m, n)[0] == 0
    # an all-zero A and an empty contraction leave C unchanged
    Cin = random_cmat(62, 2, m, n, p, 6, zero_frac=0.2)
    got, _ = _run_acc(empty_cmat(m, k, p), B, Cin, p, -1)
    assert mismatches(got, Cin, m, n)[0] == 0
    dA, dB, dC = mp.to_device(empty_cmat(m, 0, p)), mp.to_device(empty_cmat(0, n, p)), mp.to_device(Cin)
    mp.mpcg_set_stream()
    mp.mp_cgemm_acc(m, n, 0, dA, max(1, m), dB, 1, dC, dC.ld, p, -1)
    torch.cuda.synchronize()
    assert mismatches(device_result_to_host(dC, p), Cin, m, n)[0] == 0


def test_acc_large_lu_like_sampled():
    """An LU-like trailing update at 1024 bits: A22 - L21 U12 with A22 of the
    product's size, 256 x 256 x 128, checked on sampled entries."""
    p, m, n, k = 1024, 256, 256, 128
    A = random_cmat(71, 0, m, k, p, 2)
    B = random_cmat(71, 1, k, n, p, 2)
    Cin = random_cmat(71, 2, m, n, p, 6)
    got, info = _run_acc(A, B, Cin, p, -1)
    rng = np.random.default_rng(7)
    rows = np.concatenate([rng.integers(0, m, 300), [0, m - 1]])
    cols = np.concatenate([rng.integers(0, n, 300), [n - 1, 0]])
    s, e, mm = oracle.cgemm_acc_entries(A, B, Cin, rows, cols, p, -1)
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((got.re, got.im)):
            assert part.exp[j, i] == e[t, comp], (i, j, comp)
            if e[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == s[t, comp] and np.array_equal(part.mant[:, j, i], mm[t, comp])


def test_acc_truncated_bound():
    """Truncated scheme: |C~ - (Cin + sign AB)| <= 2^-(p-4) sum|a||b| + 2^-p |C~|
    (the product's truncation bound plus the one rounding of the sum)."""
    p, m, n, k = 256, 24, 20, 64
    A = random_cmat(81, 0, m, k, p, 8)
    B = random_cmat(81, 1, k, n, p, 8)
    Cin = _regime_addend(82, m, n, p, 8, base_shift=8)
    got, info = _run_acc(A, B, Cin, p, -1, M3, TRUNC)
    assert info["bound_bits"] == p - 4
    for (i, j) in [(0, 0), (3, 7), (m - 1, n - 1), (11, 2), (17, 19)]:
        scale = _absmax_terms(A, B, i, j)
        for comp, part in enumerate((got.re, got.im)):
            xn, xe = oracle.exact_entry(A, B, i, j, comp, p)
            cn, ce = oracle.entry_value(Cin.re if comp == 0 else Cin.im, i, j)
            gn, ge = oracle.entry_value(part, i, j)
            # exact = Cin - AB, all as (numerator, exponent) integers
            e0 = min(xe, ce, ge, scale[1] + 4 - p, ge - p)
            exact = (cn << (ce - e0)) - (xn << (xe - e0))
            g = gn << (ge - e0)
            rhs = (scale[0] << (scale[1] + 4 - p - e0)) + (abs(gn) << (ge - p - e0))
            assert abs(g - exact) <= rhs, (i, j, comp)


def test_acc_graph_replay_accumulates():
    """Planned from a spread bound with a caller workspace the in-place update
    is capturable; every replay applies it once more (C_n = C_{n-1} - A B,
    rounded), checked against the oracle from the previous state."""
    import torch
    import paper_2307_06072_amd as mp
    p, m, n, k, bound = 192, 40, 36, 64, 12
    A = random_cmat(91, 0, m, k, p, 6)
    B = random_cmat(91, 1, k, n, p, 6)
    C0 = random_cmat(91, 2, m, n, p, 10)
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.to_device(C0)
    opt = mp.mpcg_options(mp.MPCG_SLICE_INT8, 0, 0, 0, bound)
    wsz = mp.mpcg_workspace_size(m, n, k, p, M3, EXACT, opt, bound)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    mp.mpcg_set_workspace(ws.data_ptr(), wsz)
    try:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                mp.mpcg_set_stream(side.cuda_stream)
                mp.mp_cgemm_acc(m, n, k, dA, m, dB, k, dC, m, p, -1, M3, EXACT, max_spread=bound)
        mp.mpcg_set_stream()
        torch.cuda.synchronize()
        prev = C0
        assert mismatches(device_result_to_host(dC, p), C0, m, n)[0] == 0  # capture ran nothing
        for rep in range(3):
            dA.re.exp.add_(0)  # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = device_result_to_host(dC, p)
            ref = oracle.cgemm_acc(A, B, prev, p, -1)
            bad, first = mismatches(got, ref, m, n)
            assert bad == 0, (rep, first)
            prev = ref
        assert mp.mpcg_stream_status() == 0
    finally:
        mp.mpcg_set_workspace(None, 0)
        mp.mpcg_set_stream()


@pytest.mark.parametrize("mode", [M3, M4])
def test_batched_acc_uneven(mode):
    """The batched accumulating form: uneven problems (including empty and
    k = 0 ones), each against the oracle's once-rounded sum."""
    import torch
    import paper_2307_06072_amd as mp
    p = 190
    shapes = [(37, 45, 71), (1, 1, 1), (16, 48, 130), (50, 3, 200), (64, 64, 64), (0, 5, 5), (9, 11, 0),
              (40, 36, 400)]
    batch, devs = [], []
    for t, (m, n, k) in enumerate(shapes):
        A = random_cmat([120, t], 0, m, k, p, 8, zero_frac=0.05)
        B = random_cmat([120, t], 1, k, n, p, 8, zero_frac=0.05)
        Cin = _regime_addend(130 + t, m, n, p, 8, base_shift=8) if m and n else empty_cmat(m, n, p)
        batch.append((A, B, Cin))
        devs.append((mp.to_device(A), mp.to_device(B), mp.to_device(Cin)))
    mp.mpcg_set_stream()
    mp.mp_cgemm_batched_acc(devs, p, -1, mode)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    for t, ((A, B, Cin), (_, _, dC)) in enumerate(zip(batch, devs)):
        m, n = A.rows, B.cols
        if m == 0 or n == 0:
            continue
        got = device_result_to_host(dC, p)
        ref = Cin if A.cols == 0 else oracle.cgemm_acc(A, B, Cin, p, -1)
        bad, first = mismatches(got, ref, m, n)
        assert bad == 0, (t, shapes[t], first)


@pytest.mark.parametrize("p", [2000, 2600])
@pytest.mark.parametrize("sign", [1, -1])
def test_acc_regimes_wide_precision(sign, p):
    """Up to 2304 bits the rounding kernel keeps |X| around the addend's range
    in LDS; above that (2600 bits) it reads the product from global memory
    directly (no binary window)."""
    m, n, k = 17, 15, 24
    A = random_cmat(210, 0, m, k, p, 6, zero_frac=0.05)
    B = random_cmat(210, 1, k, n, p, 6, zero_frac=0.05)
    Cin = _regime_addend(211, m, n, p, 6, base_shift=6)
    _check(A, B, Cin, p, sign, M3)
    Rn = oracle.cgemm(A, B, p)
    _check(A, B, _flip_last_bit(Rn, p), p, -1)
