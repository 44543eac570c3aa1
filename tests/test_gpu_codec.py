"""The multi-component input codec (mpcg_from_doubles) against the oracle's
definition (the exact sum of an entry's doubles, rounded once to p bits,
ties to even), bit for bit, and the codec feeding the product."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, multi_double
from oracle import codec_ref
from tests.gpu_util import device_result_to_host, mismatches

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _device(re, im, p):
    import torch
    import paper_2307_06072_amd as mp
    mp.mpcg_set_stream()
    C = mp.from_doubles(torch.from_numpy(re).cuda(), torch.from_numpy(im).cuda(), p)
    torch.cuda.synchronize()
    st = mp.mpcg_stream_status()
    return C, device_result_to_host(C, p), st


def _zeros_are_plus(H):
    for part in (H.re, H.im):
        z = part.exp == EXP_ZERO
        assert not part.sign[z].any(), "an exact zero must be written as +0"


@pytest.mark.parametrize("p", [2, 53, 64, 107, 128, 212, 256, 1024, 2200])
@pytest.mark.parametrize("ncomp", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", ["expansion", "random", "extreme"])
def test_codec_parity(kind, ncomp, p):
    rows, cols = 23, 17  # 391 entries: four blocks of 128 threads, the last one ragged
    re = multi_double(21, 0, ncomp, rows, cols, kind, exp_range=60)
    im = multi_double(21, 1, ncomp, rows, cols, kind, exp_range=60)
    _say(f"codec kind={kind} ncomp={ncomp} p={p}")
    _, got, st = _device(re, im, p)
    assert st == 0
    ref = codec_ref.from_doubles(re, im, p)
    bad, first = mismatches(got, ref, rows, cols)
    assert bad == 0, (bad, first)
    _zeros_are_plus(got)


@pytest.mark.parametrize("kinds", [("random", "expansion"), ("extreme", "extreme")])
def test_codec_large_sampled(kinds):
    """A 1031 x 517 quad-double matrix (4166 blocks: the second pass walks it
    with a smaller grid), checked on sampled entries; the extreme inputs have
    many entries spanning more than 512 bits."""
    rows, cols, p = 1031, 517, 256
    re = multi_double(22, 0, 4, rows, cols, kinds[0], exp_range=200)
    im = multi_double(22, 1, 4, rows, cols, kinds[1], exp_range=200)
    _say("codec 1031 x 517 QD p=256")
    _, got, st = _device(re, im, p)
    assert st == 0
    rng = np.random.default_rng(5)
    rr = rng.integers(0, rows, 1500)
    cc = rng.integers(0, cols, 1500)
    for name, src in (("re", re), ("im", im)):
        sub = codec_ref.from_doubles_part(src[:, cc, rr].reshape(4, -1, 1), p)  # (ncomp, samples, 1)
        part = getattr(got, name)
        for t, (r, c) in enumerate(zip(rr, cc)):
            assert part.exp[c, r] == sub.exp[t, 0], (name, r, c)
            if sub.exp[t, 0] != EXP_ZERO:
                assert part.sign[c, r] == sub.sign[t, 0] and np.array_equal(part.mant[:, c, r], sub.mant[:, t, 0])


def test_codec_non_finite():
    import paper_2307_06072_amd as mp
    rows, cols = 5, 3
    re = multi_double(23, 0, 2, rows, cols, "expansion")
    im = multi_double(23, 1, 2, rows, cols, "expansion")
    re[1, 0, 2] = math.inf
    im[0, 2, 4] = math.nan
    _, got, st = _device(re, im, 128)
    assert st == mp.MPCG_EDOMAIN
    assert got.re.exp[0, 2] == EXP_ZERO and got.im.exp[2, 4] == EXP_ZERO
    ref = codec_ref.from_doubles(re, im, 128)
    assert mismatches(got, ref, rows, cols)[0] == 0
    assert mp.mpcg_stream_status() == 0  # the status was cleared


@pytest.mark.parametrize("mode", [0, 1])
def test_codec_feeds_the_product(mode):
    """Double-double A and B, converted on the device and multiplied, equal the
    oracle's product of the oracle's conversions."""
    import torch
    import paper_2307_06072_amd as mp
    m, k, n, p = 37, 45, 29, 212
    ar = multi_double(24, 0, 2, m, k, "expansion", 20)
    ai = multi_double(24, 1, 2, m, k, "expansion", 20)
    br = multi_double(24, 2, 2, k, n, "random", 20)
    bi = multi_double(24, 3, 2, k, n, "random", 20)
    _say(f"codec -> mp_cgemm mode={mode}")
    dA, _, st1 = _device(ar, ai, p)
    dB, _, st2 = _device(br, bi, p)
    assert st1 == 0 and st2 == 0
    dC = mp.device_empty(m, n, p)
    mp.mp_cgemm(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mode)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    got = device_result_to_host(dC, p)
    ref = oracle.cgemm(codec_ref.from_doubles(ar, ai, p), codec_ref.from_doubles(br, bi, p), p)
    bad, first = mismatches(got, ref, m, n)
    assert bad == 0, (bad, first)


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.mark.parametrize("p", [2, 53, 64, 106, 200, 256, 1024, 3000])
@pytest.mark.parametrize("ncomp", [1, 2, 3, 4])
def test_to_doubles_parity(ncomp, p):
    """Stored entries (exponents over +-1000: subnormal remainders included)
    written as ncomp doubles, against the oracle bit for bit (signed zeros
    too)."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import random_cmat
    A = random_cmat([31, p, ncomp], 0, 23, 17, p, 1000, zero_frac=0.1)
    _say(f"to_doubles p={p} ncomp={ncomp}")
    mp.mpcg_set_stream()
    re, im = mp.to_doubles(mp.to_device(A), p, ncomp)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    ref_re, ref_im = codec_ref.to_doubles(A, p, ncomp)
    assert np.array_equal(_bits(re.cpu().numpy()), _bits(ref_re))
    assert np.array_equal(_bits(im.cpu().numpy()), _bits(ref_im))


@pytest.mark.parametrize("ncomp", [2, 4])
def test_codec_round_trip(ncomp):
    """Expansions converted exactly on the device and back give themselves."""
    import torch
    import paper_2307_06072_amd as mp
    rows, cols, p = 301, 133, 64 * 4 * ncomp
    re = multi_double(32, 0, ncomp, rows, cols, "expansion", exp_range=400)
    im = multi_double(32, 1, ncomp, rows, cols, "expansion", exp_range=400)
    C, _, st = _device(re, im, p)
    assert st == 0
    bre, bim = mp.to_doubles(C, p, ncomp)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    assert np.array_equal(_bits(bre.cpu().numpy()), _bits(re))
    assert np.array_equal(_bits(bim.cpu().numpy()), _bits(im))


def test_to_doubles_overflow():
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import random_cmat, scale_exponents
    p = 128
    A = random_cmat(33, 0, 9, 7, p, 4)
    for part in (A.re, A.im):
        scale_exponents(part, rows=[0, 1], shift=1022)  # exponents 1018-1026: some beyond 2^1024
    mp.mpcg_set_stream()
    re, im = mp.to_doubles(mp.to_device(A), p, 2)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == mp.MPCG_ERANGE
    ref_re, ref_im = codec_ref.to_doubles(A, p, 2)
    assert np.isinf(ref_re).any()
    assert np.array_equal(_bits(re.cpu().numpy()), _bits(ref_re))
    assert np.array_equal(_bits(im.cpu().numpy()), _bits(ref_im))
