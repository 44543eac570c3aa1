"""Batched products and calls planned from a spread bound (no read-back,
capturable in a HIP graph), against the oracle bit for bit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, batched_inputs, random_cmat
from tests.gpu_util import device_result_to_host, mismatches

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT, TRUNC = 0, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _uneven_batch(seed, p, R, shapes):
    out = []
    for t, (m, n, k) in enumerate(shapes):
        A = random_cmat([seed, t], 0, m, k, p, R, zero_frac=0.05)
        B = random_cmat([seed, t], 1, k, n, p, R, zero_frac=0.05)
        out.append((m, n, k, A, B))
    return out


SHAPES = [(37, 45, 71), (1, 1, 1), (16, 48, 130), (50, 3, 200), (64, 64, 64), (5, 90, 17), (33, 1, 300),
          (100, 70, 9), (0, 5, 5), (7, 0, 5), (9, 11, 0), (40, 36, 400)]


def _run_batch(batch, p, mode, scheme=EXACT, **kw):
    import torch
    import paper_2307_06072_amd as mp
    devs = []
    for (m, n, k, A, B) in batch:
        dA, dB = mp.to_device(A), mp.to_device(B)
        dC = mp.device_empty(m, n, p)
        devs.append((dA, dB, dC))
    mp.mpcg_set_stream()
    info = mp.mp_cgemm_batched(devs, p, mode, scheme, **kw)
    torch.cuda.synchronize()
    st = mp.mpcg_stream_status()
    return [device_result_to_host(C, p) for (_, _, C) in devs], info, st


@pytest.mark.parametrize("mode", [M3, M4])
@pytest.mark.parametrize("p", [130, 256])
def test_batched_uneven_exact(mode, p):
    batch = _uneven_batch(60 + p, p, 8, SHAPES)
    _say(f"batched {len(batch)} problems p={p} mode={mode}")
    res, info, st = _run_batch(batch, p, mode)
    assert st == 0
    for t, ((m, n, k, A, B), C) in enumerate(zip(batch, res)):
        if m == 0 or n == 0:
            continue
        if k == 0:  # empty contraction: +0 everywhere
            assert (C.re.exp[:n, :m] == EXP_ZERO).all() and (C.im.exp[:n, :m] == EXP_ZERO).all()
            continue
        R = oracle.cgemm(A, B, p)
        bad, first = mismatches(C, R, m, n)
        assert bad == 0, (t, (m, n, k), first, info)


@pytest.mark.parametrize("block", [8, 12, 16, 20])
@pytest.mark.parametrize("ksplit", [0, 3])
def test_batched_plan_independent(block, ksplit):
    p = 200
    batch = _uneven_batch(71, p, 6, [(40, 36, 300), (17, 70, 130), (64, 32, 64)])
    res, info, st = _run_batch(batch, p, M3, block_override=block, ksplit_override=ksplit)
    assert st == 0 and info["block"] == block
    for (m, n, k, A, B), C in zip(batch, res):
        bad, first = mismatches(C, oracle.cgemm(A, B, p), m, n)
        assert bad == 0, (block, ksplit, first)


def test_batched_spread_bound():
    """Planned from a spread bound (no read-back) the bits are unchanged, and a
    bound below the data's spread is reported."""
    p = 256
    batch = _uneven_batch(72, p, 8, [(30, 20, 50), (64, 48, 100), (9, 70, 33)])
    res, info, st = _run_batch(batch, p, M3, max_spread=16)
    assert st == 0
    for (m, n, k, A, B), C in zip(batch, res):
        bad, first = mismatches(C, oracle.cgemm(A, B, p), m, n)
        assert bad == 0, first
    # a bound below the data's spread is reported
    _, _, st = _run_batch(batch, p, M3, max_spread=5)
    import paper_2307_06072_amd as mp
    assert st == mp.MPCG_ESPREAD


def test_batched_config_256_uneven_sampled():
    """The 256-problem family (shapes uniform on [16, 768], 256 bits): every
    problem checked on sampled entries."""
    p = 256
    batch = batched_inputs(256, 4, p, 8)
    _say("batched config: 256 problems")
    res, info, st = _run_batch(batch, p, M3)
    assert st == 0
    _say(f"  S_A<={info['S_A']} pairs={info['pairs']} block={info['block']}")
    rng = np.random.default_rng(8)
    for t, ((m, n, k, A, B), C) in enumerate(zip(batch, res)):
        rows = np.concatenate([rng.integers(0, m, 6), [0, m - 1]])
        cols = np.concatenate([rng.integers(0, n, 6), [n - 1, 0]])
        s, e, mm = oracle.cgemm_entries(A, B, rows, cols, p)
        for u, (i, j) in enumerate(zip(rows, cols)):
            for comp, part in enumerate((C.re, C.im)):
                assert part.exp[j, i] == e[u, comp], (t, i, j, comp)
                if e[u, comp] != EXP_ZERO:
                    assert part.sign[j, i] == s[u, comp] and np.array_equal(part.mant[:, j, i], mm[u, comp])


def test_single_call_spread_bound_graph_replay():
    """A call planned from a spread bound with a caller workspace allocates and
    synchronizes nothing, so it can be captured; every replay (with eager work
    and synchronizations in between) reproduces the eager result."""
    import torch
    import paper_2307_06072_amd as mp
    p, m, n, k, bound = 192, 48, 40, 96, 20
    A = random_cmat(81, 0, m, k, p, 8)
    B = random_cmat(81, 1, k, n, p, 8)
    ref = oracle.cgemm(A, B, p)
    dA, dB = mp.to_device(A), mp.to_device(B)
    opt = mp.mpcg_options(mp.MPCG_SLICE_INT8, 0, 0, 0, bound)
    wsz = mp.mpcg_workspace_size(m, n, k, p, M3, EXACT, opt, bound)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    mp.mpcg_set_workspace(ws.data_ptr(), wsz)
    try:
        C0 = mp.device_empty(m, n, p)
        mp.mpcg_set_stream()
        mp.mp_cgemm_ex(m, n, k, dA, m, dB, k, C0, m, p, M3, EXACT, max_spread=bound)
        torch.cuda.synchronize()
        assert mp.mpcg_stream_status() == 0
        eager = device_result_to_host(C0, p)
        assert mismatches(eager, ref, m, n)[0] == 0
        C = mp.device_empty(m, n, p)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                mp.mpcg_set_stream(side.cuda_stream)
                mp.mp_cgemm_ex(m, n, k, dA, m, dB, k, C, m, p, M3, EXACT, max_spread=bound)
        torch.cuda.synchronize()
        for rep in range(3):
            for part in (C.re, C.im):  # clobber the output between replays
                part.exp.fill_(7)
                part.mant.fill_(0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = device_result_to_host(C, p)
            bad, first = mismatches(got, eager, m, n)
            assert bad == 0, (rep, first)
        mp.mpcg_set_stream()
        assert mp.mpcg_stream_status() == 0
    finally:
        mp.mpcg_set_workspace(None, 0)
        mp.mpcg_set_stream()


def test_batched_spread_bound_graph_replay():
    """A batch planned from a spread bound with a caller workspace of
    mpcg_workspace_size_batched bytes, captured once, replayed three times
    with other batched and single calls in between (they rewrite and regrow
    the library's own staging and table buffers): every replay gives the
    oracle's bits."""
    import torch
    import paper_2307_06072_amd as mp
    p, R, bound = 256, 6, 12
    shapes = [(37, 45, 71), (16, 48, 130), (50, 3, 200), (64, 64, 64), (5, 90, 17), (100, 70, 9), (1, 1, 1)]
    batch = _uneven_batch(95, p, R, shapes)
    refs = [oracle.cgemm(A, B, p) for (m, n, k, A, B) in batch]
    devs = [(mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)) for (m, n, k, A, B) in batch]
    mp.mpcg_set_stream()
    mp.mp_cgemm_batched(devs, p, M3, EXACT, max_spread=bound)  # eager, also sets up the library
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    wsz = mp.mpcg_workspace_size_batched(devs, p, M3, EXACT, max_spread=bound)
    assert wsz > 0
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    _say("batched capture")
    mp.mpcg_set_workspace(ws.data_ptr(), wsz)
    try:
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                mp.mpcg_set_stream(side.cuda_stream)
                mp.mp_cgemm_batched(devs, p, M3, EXACT, max_spread=bound)
    finally:
        mp.mpcg_set_workspace(None, 0)
        mp.mpcg_set_stream()
    torch.cuda.synchronize()
    other = _uneven_batch(96, 200, 4, [(70, 80, 90), (120, 33, 60), (9, 9, 300)])
    for rep in range(3):
        for (_, _, C) in devs:
            for part in (C.re, C.im):
                part.exp.fill_(7)
                part.mant.fill_(0)
        res, _, st = _run_batch(other[: 1 + rep], 200, M3)  # library tables rewritten (and grown)
        assert st == 0
        for (m, n, k, A, B), C in zip(other[: 1 + rep], res):
            assert mismatches(C, oracle.cgemm(A, B, 200), m, n)[0] == 0
        torch.cuda.synchronize()
        _say(f"batched replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert mp.mpcg_stream_status() == 0
        for t, ((m, n, k, A, B), (_, _, C)) in enumerate(zip(batch, devs)):
            bad, first = mismatches(device_result_to_host(C, p), refs[t], m, n)
            assert bad == 0, (rep, t, first)
