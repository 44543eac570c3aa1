"""Adaptive slicing (mpcg_options.adaptive): slice counts per block of rows of
A and of columns of B.  Exact-scheme bits equal the single-plan call and the
oracle; less slice-pair work where the blocks' spreads differ; the truncated
bound still holds."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, random_cmat
from tests.gpu_util import mismatches, run_device
from tests.test_gpu_truncated import _check_bound

pytestmark = pytest.mark.gpu

M3, M4, EXACT, I8 = 1, 0, 0, 0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_sampled(C, A, B, p, rows, cols, Cin=None, sign=1):
    """C's entries (rows[t], cols[t]) against the oracle's, bit for bit (the
    accumulating form's when Cin is given)."""
    if Cin is None:
        sg, ex, mt = oracle.cgemm_entries(A, B, rows, cols, p)
    else:
        sg, ex, mt = oracle.cgemm_acc_entries(A, B, Cin, rows, cols, p, sign)
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((C.re, C.im)):
            assert part.exp[j, i] == ex[t, comp], (i, j, comp)
            if ex[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == sg[t, comp] and np.array_equal(part.mant[:, j, i], mt[t, comp]), \
                    (i, j, comp)


def _mixed(m, n, k, p, shift, seed=61):
    """Random A (m x k) and B (k x n); rows 256..511 of A and columns 256.. of B
    get one entry each raised by 2^shift, so those rows' and columns' exponent
    spreads grow by `shift` bits while the others keep theirs."""
    A = random_cmat([seed, m, n, k], 0, m, k, p, 8)
    B = random_cmat([seed, m, n, k], 1, k, n, p, 8)
    for r in range(256, min(m, 512)):
        if A.re.exp[3, r] != EXP_ZERO:
            A.re.exp[3, r] += np.int32(shift)
    for c in range(256, n):
        if B.re.exp[c, 5] != EXP_ZERO:
            B.re.exp[c, 5] += np.int32(shift)
    return A, B


@pytest.mark.parametrize("mode", [M3, M4])
def test_adaptive_exact_bits_and_pairs(mode):
    m, n, k, p = 600, 300, 70, 256
    A, B = _mixed(m, n, k, p, 150)
    _say(f"adaptive exact m={m} n={n} k={k} mode={mode}")
    C0, info0 = run_device(A, B, p, mode, EXACT, I8)
    C1, info1 = run_device(A, B, p, mode, EXACT, I8, adaptive=1)
    assert mismatches(C1, C0, m, n)[0] == 0
    assert info1["algo_ops"] < 0.8 * info0["algo_ops"], (info0, info1)  # fewer slice pairs where spreads are small
    rng = np.random.default_rng(7)
    rows, cols = rng.integers(0, m, 300), rng.integers(0, n, 300)
    sg, ex, mt = oracle.cgemm_entries(A, B, rows, cols, p)
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((C1.re, C1.im)):
            assert part.exp[j, i] == ex[t, comp]
            if ex[t, comp] != EXP_ZERO:
                assert part.sign[j, i] == sg[t, comp] and np.array_equal(part.mant[:, j, i], mt[t, comp])


def test_adaptive_uniform_input_is_one_plan():
    m = n = k = 300
    p = 128
    A = random_cmat([62], 0, m, k, p, 8)
    B = random_cmat([62], 1, k, n, p, 8)
    C0, info0 = run_device(A, B, p, M3, EXACT, I8)
    C1, info1 = run_device(A, B, p, M3, EXACT, I8, adaptive=1)
    assert info0 == info1
    assert mismatches(C1, C0, m, n)[0] == 0
    rng = np.random.default_rng(62)
    _oracle_sampled(C1, A, B, p, rng.integers(0, m, 150), rng.integers(0, n, 150))


def test_adaptive_truncated_bound():
    m, n, k, p = 520, 280, 40, 192
    A, B = _mixed(m, n, k, p, 120, seed=63)
    rng = np.random.default_rng(8)
    entries = list(zip(rng.integers(0, m, 60), rng.integers(0, n, 60))) + [(300, 270), (10, 10), (519, 279)]
    info, _ = _check_bound(A, B, p, M3, I8, entries, adaptive=1)


def test_adaptive_accumulate_matches_single_plan():
    import torch
    import paper_2307_06072_amd as mp
    m, n, k, p = 530, 290, 33, 256
    A, B = _mixed(m, n, k, p, 100, seed=64)
    Cin = random_cmat([64], 2, m, n, p, 8)
    outs = []
    for adaptive in (0, 1):
        dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.to_device(Cin)
        mp.mpcg_set_stream()
        mp.mp_cgemm_acc(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, -1, adaptive=adaptive)
        torch.cuda.synchronize()
        assert mp.mpcg_stream_status() == 0
        from tests.gpu_util import device_result_to_host
        outs.append(device_result_to_host(dC, p))
    assert mismatches(outs[1], outs[0], m, n)[0] == 0
    rng = np.random.default_rng(64)
    rows = np.concatenate([rng.integers(0, m, 150), [0, 255, 256, 511, 529]])
    cols = np.concatenate([rng.integers(0, n, 150), [0, 255, 256, 289, 289]])
    _oracle_sampled(outs[1], A, B, p, rows, cols, Cin=Cin, sign=-1)


def test_adaptive_block_size():
    """Wide rows 64..127 only: blocks of 64 confine them, blocks of 256 widen
    rows 0..255; the bits stay those of the single plan."""
    m, n, k, p = 300, 200, 40, 192
    A = random_cmat([65], 0, m, k, p, 8)
    B = random_cmat([65], 1, k, n, p, 8)
    for r in range(64, 128):
        if A.re.exp[2, r] != EXP_ZERO:
            A.re.exp[2, r] += np.int32(200)
    C0, info0 = run_device(A, B, p, M3, EXACT, I8)
    C1, info1 = run_device(A, B, p, M3, EXACT, I8, adaptive=1)
    C2, info2 = run_device(A, B, p, M3, EXACT, I8, adaptive=64)
    assert mismatches(C1, C0, m, n)[0] == 0 and mismatches(C2, C0, m, n)[0] == 0
    assert info2["algo_ops"] < info1["algo_ops"] < info0["algo_ops"], (info0, info1, info2)
    rng = np.random.default_rng(65)
    rows = np.concatenate([rng.integers(0, m, 120), np.arange(60, 132, 4)])
    cols = np.concatenate([rng.integers(0, n, 120), rng.integers(0, n, 18)])
    _oracle_sampled(C2, A, B, p, rows, cols)
