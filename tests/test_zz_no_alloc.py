"""mp_cgemm_ex_noalloc (every scratch byte from the library's fixed device
buffer) against mp_cgemm_ex and the oracle, bit for bit, through the C-ABI:
two calls in a row, the second smaller; the capturable form (spread bound)
replayed from a HIP graph; a product too large for the buffer rejected."""
from __future__ import annotations

import sys

import pytest

import oracle
from mpgen import EXP_ZERO, random_cmat
from tests.gpu_util import device_result_to_host, mismatches

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT, TRUNC = 0, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(m, n, k, p, R, seed, mode, scheme, bound=0):
    """(noalloc result, mp_cgemm_ex result, oracle) of one product."""
    import torch
    import paper_2307_06072_amd as mp
    A = random_cmat([seed, m, k], 0, m, k, p, R, zero_frac=0.05)
    B = random_cmat([seed, m, k], 1, k, n, p, R, zero_frac=0.05)
    dA, dB = mp.to_device(A), mp.to_device(B)
    mp.mpcg_set_stream()
    C1 = mp.device_empty(m, n, p)
    info1 = mp.mp_cgemm_ex_noalloc(m, n, k, dA, m, dB, k, C1, m, p, mode, scheme, max_spread=bound)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0, mp.mpcg_last_error()
    C2 = mp.device_empty(m, n, p)
    info2 = mp.mp_cgemm_ex(m, n, k, dA, m, dB, k, C2, m, p, mode, scheme, max_spread=bound)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0, mp.mpcg_last_error()
    assert info1 == info2
    return device_result_to_host(C1, p), device_result_to_host(C2, p), A, B


@pytest.mark.parametrize("mode,scheme,bound", [(M3, EXACT, 0), (M4, EXACT, 0), (M3, TRUNC, 0), (M3, EXACT, 24)])
def test_two_calls_second_smaller(mode, scheme, bound):
    for (m, n, k, p, R) in [(150, 131, 200, 256, 10), (37, 20, 65, 130, 6)]:
        _say(f"noalloc m={m} n={n} k={k} p={p} mode={mode} scheme={scheme} bound={bound}")
        got, ex, A, B = _both(m, n, k, p, R, 91, mode, scheme, bound)
        bad, first = mismatches(got, ex, m, n)
        assert bad == 0, (first,)
        if scheme == EXACT:
            bad, first = mismatches(got, oracle.cgemm(A, B, p), m, n)
            assert bad == 0, (first,)


def test_graph_replay_with_spread_bound():
    """Captured once, replayed three times with other work in between (another
    product through the same buffer): every replay matches the eager call."""
    import torch
    import paper_2307_06072_amd as mp
    p, m, n, k, bound = 192, 48, 40, 96, 20
    A = random_cmat(83, 0, m, k, p, 8)
    B = random_cmat(83, 1, k, n, p, 8)
    ref = oracle.cgemm(A, B, p)
    dA, dB = mp.to_device(A), mp.to_device(B)
    mp.mpcg_set_stream()
    C0 = mp.device_empty(m, n, p)
    mp.mp_cgemm_ex_noalloc(m, n, k, dA, m, dB, k, C0, m, p, M3, EXACT, max_spread=bound)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    assert mismatches(device_result_to_host(C0, p), ref, m, n)[0] == 0
    C = mp.device_empty(m, n, p)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    _say("noalloc capture")
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
            mp.mpcg_set_stream(side.cuda_stream)
            mp.mp_cgemm_ex_noalloc(m, n, k, dA, m, dB, k, C, m, p, M3, EXACT, max_spread=bound)
    torch.cuda.synchronize()
    mp.mpcg_set_stream()
    for rep in range(3):
        for part in (C.re, C.im):
            part.exp.fill_(7)
            part.mant.fill_(0)
        # other work through the same buffer between replays
        got_other, ex_other, _, _ = _both(30, 22, 50, 128, 4, 84 + rep, M3, EXACT)
        assert mismatches(got_other, ex_other, 30, 22)[0] == 0
        torch.cuda.synchronize()
        _say(f"noalloc replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        bad, first = mismatches(device_result_to_host(C, p), ref, m, n)
        assert bad == 0, (rep, first)
    assert mp.mpcg_stream_status() == 0


def test_too_large_is_rejected():
    """A product whose workspace exceeds the buffer returns MPCG_ENOMEM and
    leaves C untouched; the next call still works."""
    import torch
    import paper_2307_06072_amd as mp
    m = n = k = 1024
    p = 1024
    dA = mp.device_empty(m, k, p)
    dB = mp.device_empty(k, n, p)
    C = mp.device_empty(m, n, p)
    for part in (C.re, C.im):
        part.exp.fill_(5)
    mp.mpcg_set_stream()
    a, b, c = dA.struct(), dB.struct(), C.struct()
    import ctypes
    opt = mp.mpcg_options(mp.MPCG_SLICE_INT8, 0, 0, 0, 64)
    rc = mp.mp_cgemm_ex_noalloc_raw(m, n, k, ctypes.byref(a), m, ctypes.byref(b), k, ctypes.byref(c), m, p, M3,
                                    EXACT, ctypes.byref(opt), None)
    assert rc == mp.MPCG_ENOMEM, rc
    assert "fixed buffer" in mp.mpcg_last_error()
    torch.cuda.synchronize()
    assert int((C.re.exp != 5).sum()) == 0
    got, ex, _, _ = _both(20, 20, 20, 64, 3, 85, M3, EXACT)
    assert mismatches(got, ex, 20, 20)[0] == 0


def test_products_apart_fall_back_to_fused():
    """A 3M product that mp_cgemm_ex runs with its real products apart (three
    digit streams per contraction chunk, about 153 MiB of workspace here)
    while its fused plan fits the buffer: this entry point runs the products
    together and gives the same bits, which the oracle confirms on samples."""
    import numpy as np
    import torch
    import paper_2307_06072_amd as mp
    m = n = 256
    k, p = 640, 256
    _say(f"noalloc fallback m={m} n={n} k={k} p={p}")
    A = random_cmat([93, m, k], 0, m, k, p, 2)
    B = random_cmat([93, m, k], 1, k, n, p, 2)
    dA, dB = mp.to_device(A), mp.to_device(B)
    mp.mpcg_set_stream()
    C1 = mp.device_empty(m, n, p)
    info1 = mp.mp_cgemm_ex_noalloc(m, n, k, dA, m, dB, k, C1, m, p, M3, EXACT)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0, mp.mpcg_last_error()
    C2 = mp.device_empty(m, n, p)
    info2 = mp.mp_cgemm_ex(m, n, k, dA, m, dB, k, C2, m, p, M3, EXACT)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0, mp.mpcg_last_error()
    assert info2["apart"] == 1 and info1["apart"] == 0, (info1, info2)
    got, ex = device_result_to_host(C1, p), device_result_to_host(C2, p)
    bad, first = mismatches(got, ex, m, n)
    assert bad == 0, (first,)
    rng = np.random.default_rng(5)
    rows = np.concatenate([rng.integers(0, m, 200), [0, m - 1]])
    cols = np.concatenate([rng.integers(0, n, 200), [n - 1, 0]])
    s, e, mm = oracle.cgemm_entries(A, B, rows, cols, p)
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((got.re, got.im)):
            assert part.exp[j, i] == e[t, comp], (i, j, comp)
            if e[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == s[t, comp]
                assert np.array_equal(part.mant[:, j, i], mm[t, comp])
