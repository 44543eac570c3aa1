"""Full-size workloads (2048 x 2048 x 2048 at 1024 bits, in the launch
configuration the benchmark times) checked on sampled entries against the
oracle, plus determinism and the device-detected error statuses."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import EXP_ZERO, random_cmat, workload_inputs
from tests.gpu_util import mismatches, run_device
from tests.test_gpu_truncated import _check_bound

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT, TRUNC = 0, 1
I8, F64 = 0, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sample(m, n, seed, count, rows=(), cols=()):
    rng = np.random.default_rng(seed)
    ri = list(rng.integers(0, m, count))
    ci = list(rng.integers(0, n, count))
    for r in rows:  # whole rows at a few columns and whole columns at a few rows
        for c in list(range(0, n, max(1, n // 64))) + [n - 1]:
            ri.append(r)
            ci.append(c)
    for c in cols:
        for r in list(range(0, m, max(1, m // 64))) + [m - 1]:
            ri.append(r)
            ci.append(c)
    return np.array(ri, np.int64), np.array(ci, np.int64)


def _check_sampled(C, rows, cols, s, e, mm, what):
    bad = 0
    first = None
    for t, (i, j) in enumerate(zip(rows, cols)):
        for comp, part in enumerate((C.re, C.im)):
            ok = part.exp[j, i] == e[t, comp]
            if ok and e[t, comp] != EXP_ZERO:
                ok = part.sign[j, i] == s[t, comp] and np.array_equal(part.mant[:, j, i], mm[t, comp])
            if not ok:
                bad += 1
                first = first or (int(i), int(j), comp)
    assert bad == 0, f"{what}: {bad} mismatching sampled components, first {first}"


@pytest.mark.parametrize("workload,rows,cols", [
    ("cgemm2048_p1024", (0, 2047), (0, 2047)),
    ("cgemm2048_p1024_rowcol60", (7,), (11,)),       # row 7 of A and column 11 of B scaled by 2^60
    ("cgemm2048_p1024_contract60", (0,), (0,)),     # column 7 of A and row 7 of B scaled by 2^60
])
def test_config_2048_p1024_sampled(workload, rows, cols):
    m, n, k, p, A, B = workload_inputs(workload)
    ri, ci = _sample(m, n, 3, 1500, rows, cols)
    _say(f"{workload}: oracle on {ri.size} entries")
    s, e, mm = oracle.cgemm_entries(A, B, ri, ci, p)
    _say(f"{workload}: device 3M exact (default plan)")
    C, info = run_device(A, B, p, M3, EXACT, I8)
    _say(f"  S_A={info['S_A']} S_B={info['S_B']} pairs={info['pairs']} ksplit={info['ksplit']} block={info['block']}")
    _check_sampled(C, ri, ci, s, e, mm, workload)
    if workload == "cgemm2048_p1024_contract60":
        # the scaled contraction index widens every row's spread by 60 bits:
        # more slices than the 1024 + 3 + 64 bits of the unscaled workload need
        assert info["S_A"] * info["w"] > 1024 + 3 + 64 + 48


def test_config_2048_p1024_4m_and_truncated():
    m, n, k, p, A, B = workload_inputs("cgemm2048_p1024")
    ri, ci = _sample(m, n, 4, 600)
    s, e, mm = oracle.cgemm_entries(A, B, ri, ci, p)
    _say("cgemm2048_p1024: device 4M exact")
    C, info = run_device(A, B, p, M4, EXACT, I8)
    _check_sampled(C, ri, ci, s, e, mm, "4M exact")
    entries = list(zip(ri[:12].tolist(), ci[:12].tolist()))
    info, _ = _check_bound(A, B, p, M3, I8, entries)
    _say(f"  truncated 3M: cutoff {info['cutoff']} pairs {info['pairs']}")


def test_deterministic_and_forms_agree():
    """Exact mode: repeated calls, 3M/4M and INT8/FP64 give identical bits."""
    m, n, k, p = 70, 66, 150, 300
    A = random_cmat(9, 0, m, k, p, 12, zero_frac=0.05)
    B = random_cmat(9, 1, k, n, p, 12, zero_frac=0.05)
    ref, _ = run_device(A, B, p, M3, EXACT, I8)
    for mode, st in [(M3, I8), (M4, I8), (M4, F64), (M3, F64)]:
        C, _ = run_device(A, B, p, mode, EXACT, st)
        bad, first = mismatches(C, ref, m, n)
        assert bad == 0, (mode, st, first)


def test_input_exponent_out_of_range():
    import paper_2307_06072_amd as mp
    p = 64
    A = random_cmat(12, 0, 4, 4, p, 2)
    B = random_cmat(12, 1, 4, 4, p, 2)
    A.re.exp[2, 1] = (1 << 30) + 1
    with pytest.raises(mp.MPCGError) as ex:
        run_device(A, B, p, M3, EXACT)
    assert ex.value.code == mp.MPCG_ERANGE


def test_output_exponent_overflow_status():
    """Products of exponents near 2^30 overflow int32: those entries read +0 and
    the stream status reports ERANGE; the other entries are still correct."""
    import torch
    import paper_2307_06072_amd as mp
    p, m, n, k = 64, 4, 4, 4
    A = random_cmat(13, 0, m, k, p, 2)
    B = random_cmat(13, 1, k, n, p, 2)
    A.im.exp[:, 0] = EXP_ZERO
    A.re.sign[:, 0] = 0
    A.re.exp[:, 0] = 1 << 30  # row 0 of A: large positive real entries
    B.im.exp[0, :] = EXP_ZERO
    B.re.sign[0, :] = 0
    B.re.exp[0, :] = 1 << 30  # column 0 of B likewise
    dA, dB = mp.to_device(A), mp.to_device(B)
    C, _ = mp.matmul(dA, dB, p, mode=M3)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == mp.MPCG_ERANGE
    assert mp.mpcg_stream_status() == mp.MPCG_OK  # cleared
    from tests.gpu_util import device_result_to_host
    H = device_result_to_host(C, p)
    assert H.re.exp[0, 0] == EXP_ZERO
    R = oracle.cgemm_entries(A, B, [1, 2, 3], [1, 2, 3], p)
    for t, i in enumerate([1, 2, 3]):
        assert H.re.exp[i, i] == R[1][t, 0] and H.im.exp[i, i] == R[1][t, 1]


def test_unnormalized_input_status():
    import torch
    import paper_2307_06072_amd as mp
    p = 64
    A = random_cmat(14, 0, 4, 4, p, 2)
    B = random_cmat(14, 1, 4, 4, p, 2)
    A.re.mant[0, 1, 2] &= np.uint64(0x7FFFFFFFFFFFFFFF)  # clear the top bit of a nonzero entry
    A.re.exp[1, 2] = 3
    dA, dB = mp.to_device(A), mp.to_device(B)
    mp.matmul(dA, dB, p, mode=M3)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == mp.MPCG_EDOMAIN


def test_acc_full_size_update_sampled():
    """The accumulating form at full size: a 2048 x 2048 x 128 update
    C := C - A B at 1024 bits (an LU trailing update of the 2048 family's
    precision), checked on sampled entries against the oracle."""
    import torch
    import paper_2307_06072_amd as mp
    p, m, n, k = 1024, 2048, 2048, 128
    A = random_cmat(33, 0, m, k, p, 8)
    B = random_cmat(33, 1, k, n, p, 8)
    Cin = random_cmat(33, 2, m, n, p, 12)
    ri, ci = _sample(m, n, 5, 400, rows=(0, m - 1), cols=(n - 1,))
    _say(f"acc 2048x2048x128 p=1024: oracle on {ri.size} entries")
    s, e, mm = oracle.cgemm_acc_entries(A, B, Cin, ri, ci, p, -1)
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.to_device(Cin)
    mp.mpcg_set_stream()
    mp.mp_cgemm_acc(m, n, k, dA, m, dB, k, dC, m, p, -1, M3, EXACT)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    from tests.gpu_util import device_result_to_host
    _check_sampled(device_result_to_host(dC, p), ri, ci, s, e, mm, "acc 2048")
