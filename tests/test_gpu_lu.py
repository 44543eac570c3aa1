"""The blocked complex LU (mp_zgetrf) and its solve (mp_zgetrs) against the
oracle's step-by-step mirror (oracle/lu_ref.py), bit for bit, and against
closed forms: factors known exactly, and the paper's problem b = A x with
x_k = k + k i solved to a tiny relative error."""
from __future__ import annotations

import sys
from fractions import Fraction

import numpy as np
import pytest

from mpgen import random_cmat
from oracle import lu_ref
from oracle.fraction_ref import decode
from tests.gpu_util import device_result_to_host, mismatches
from tests.lu_cases import column, diagonal_pivots, dominant_matrix, exact_case, to_cmat

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _factor(A, nb, p, mode):
    import torch
    import paper_2307_06072_amd as mp
    mp.mpcg_set_stream()
    n = A.rows
    dA = mp.to_device(A)
    ipiv = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
    info = mp.mp_zgetrf(n, dA, dA.ld, ipiv, nb, p, mode)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    return dA, ipiv, info


@pytest.mark.parametrize("n,nb,p,mode", [(1, 1, 64, 1), (2, 1, 64, 0), (5, 2, 128, 1), (17, 8, 256, 1),
                                         (40, 16, 256, 1), (33, 64, 128, 0), (24, 5, 1000, 1), (9, 4, 2, 1),
                                         (6, 4, 4096, 1), (65, 64, 128, 1), (200, 128, 256, 1),
                                         (150, 128, 192, 0)])
def test_getrf_parity(n, nb, p, mode):
    A = random_cmat([51, n, p], 0, n, n, p, 2)
    _say(f"getrf n={n} nb={nb} p={p} mode={mode}")
    dA, ipiv, info = _factor(A, nb, p, mode)
    ref, ref_piv, ref_info = lu_ref.getrf(A, nb, p)
    assert info == ref_info
    assert np.array_equal(ipiv.cpu().numpy()[:n], ref_piv)
    bad, first = mismatches(device_result_to_host(dA, p), ref, n, n)
    assert bad == 0, (bad, first)


@pytest.mark.parametrize("n,nrhs,nb,p", [(17, 3, 8, 256), (6, 1, 2, 64), (5, 2, 3, 4096)])
def test_getrs_parity(n, nrhs, nb, p):
    import torch
    import paper_2307_06072_amd as mp
    A = random_cmat([52, n, p], 0, n, n, p, 2)
    B = random_cmat([52, n, p], 1, n, nrhs, p, 2)
    _say(f"getrs n={n} nrhs={nrhs} p={p}")
    dA, ipiv, info = _factor(A, nb, p, 1)
    dB = mp.to_device(B)
    mp.mp_zgetrs(n, nrhs, dA, dA.ld, ipiv, dB, dB.ld, p, 1)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    LU, piv, _ = lu_ref.getrf(A, nb, p)
    ref = lu_ref.getrs(LU, piv, B, p)
    bad, first = mismatches(device_result_to_host(dB, p), ref, n, nrhs)
    assert bad == 0, (bad, first)


def test_exact_factors_n64():
    """Closed-form factors at n = 64 (four block columns of 16): L, U, the
    interchanges and the solution x_k = k + k i come back exactly."""
    import torch
    import paper_2307_06072_amd as mp
    n, nb, p = 64, 16, 256
    case = exact_case(n, seed=5)
    _say("getrf exact n=64")
    dA, ipiv, info = _factor(to_cmat(case["A"], p), nb, p, 1)
    assert info == 0
    assert np.array_equal(ipiv.cpu().numpy(), case["ipiv"])
    F = device_result_to_host(dA, p)
    for i in range(n):
        for j in range(n):
            assert (decode(F.re, i, j, p), decode(F.im, i, j, p)) == case["packed"][i][j], (i, j)
    dB = mp.to_device(to_cmat(column(case["b"]), p))
    mp.mp_zgetrs(n, 1, dA, dA.ld, ipiv, dB, dB.ld, p, 1)
    torch.cuda.synchronize()
    X = device_result_to_host(dB, p)
    assert [(decode(X.re, i, 0, p), decode(X.im, i, 0, p)) for i in range(n)] == case["x"]


def test_paper_problem_n256():
    """The paper's LU experiment at n = 256, 256 bits, K = 64: b = A x with
    x_k = k + k i (b rounded once at 256 bits), solved through the factors;
    the relative error of x is a few units of 2^-256 times the condition."""
    import torch
    import paper_2307_06072_amd as mp
    n, nb, p = 256, 64, 256
    A = random_cmat([53, n, p], 0, n, n, p, 2)
    x = [(Fraction(k + 1), Fraction(k + 1)) for k in range(n)]
    dA = mp.to_device(A)
    dx = mp.to_device(to_cmat(column(x), p))
    dB = mp.device_empty(n, 1, p)
    mp.mpcg_set_stream()
    mp.mp_cgemm(n, 1, n, dA, dA.ld, dx, dx.ld, dB, dB.ld, p)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    _say("getrf + getrs n=256 p=256")
    assert mp.mp_zgetrf(n, dA, dA.ld, ipiv, nb, p, 1) == 0
    mp.mp_zgetrs(n, 1, dA, dA.ld, ipiv, dB, dB.ld, p, 1)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    X = device_result_to_host(dB, p)
    err = max((abs(decode(X.re, k, 0, p) - x[k][0]) + abs(decode(X.im, k, 0, p) - x[k][1])) / (2 * x[k][0])
              for k in range(n))
    _say(f"max relative error {float(err):.3e}")
    assert err < Fraction(2) ** (32 - p)


def test_zero_pivot_info():
    p = 64
    one, zero = Fraction(1), Fraction(0)
    vals = [[(one, zero), (zero, zero), (one, one)],
            [(Fraction(1, 2), zero), (zero, zero), (zero, one)],
            [(zero, one), (zero, zero), (one, zero)]]
    A = to_cmat(vals, p)
    dA, ipiv, info = _factor(A, 2, p, 1)
    ref, ref_piv, ref_info = lu_ref.getrf(A, 2, p)
    assert info == ref_info == 2
    assert np.array_equal(ipiv.cpu().numpy(), ref_piv)
    assert mismatches(device_result_to_host(dA, p), ref, 3, 3)[0] == 0


def test_reciprocal_chain_wide_exponents():
    """Pivots far from 1 (exponents +-500) keep the parity."""
    n, nb, p = 12, 5, 320
    A = random_cmat([54, n, p], 0, n, n, p, 500)
    _say("getrf wide exponents")
    dA, ipiv, info = _factor(A, nb, p, 1)
    ref, ref_piv, ref_info = lu_ref.getrf(A, nb, p)
    assert info == ref_info and np.array_equal(ipiv.cpu().numpy(), ref_piv)
    bad, first = mismatches(device_result_to_host(dA, p), ref, n, n)
    assert bad == 0, (bad, first)


def _rhs_ones(A, n, p):
    """b = A (1 + i) ones, rounded once (the oracle's product)."""
    import oracle
    ones = to_cmat(column([(Fraction(1), Fraction(1))] * n), p)
    return oracle.cgemm(A, ones, p)


def test_dominant_n256_nb128():
    """The factorization workload at the size the oracle checks: A random
    (exponents on [-2, 2]) plus 256 (1 + i) on the diagonal, block width 128,
    256 bits; b = A (1 + i) ones.  Factors, interchanges and solution are
    bit-identical to the oracle's, and x is (1 + i) ones to a few units of
    2^-256."""
    import torch
    import paper_2307_06072_amd as mp
    n, nb, p = 256, 128, 256
    A = dominant_matrix(n, p, [5, n])
    b = _rhs_ones(A, n, p)
    _say("getrf dominant n=256 nb=128 p=256")
    dA, ipiv, info = _factor(A, nb, p, 1)
    ref, ref_piv, ref_info = lu_ref.getrf(A, nb, p)
    assert info == ref_info == 0
    assert np.array_equal(ipiv.cpu().numpy()[:n], ref_piv)
    bad, first = mismatches(device_result_to_host(dA, p), ref, n, n)
    assert bad == 0, (bad, first)
    _say("getrs dominant n=256")
    dB = mp.to_device(b)
    mp.mp_zgetrs(n, 1, dA, dA.ld, ipiv, dB, dB.ld, p, 1)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    refx = lu_ref.getrs(ref, ref_piv, b, p)
    X = device_result_to_host(dB, p)
    bad, first = mismatches(X, refx, n, 1)
    assert bad == 0, (bad, first)
    err = max(abs(decode(X.re, k, 0, p) - 1) + abs(decode(X.im, k, 0, p) - 1) for k in range(n)) / 2
    _say(f"max relative error {float(err):.3e}")
    assert err < Fraction(2) ** (8 - p)


@pytest.mark.parametrize("n,p", [(64, 256), (48, 53), (40, 1024), (16, 2), (24, 100), (8, 4096)])
def test_reciprocals_correctly_rounded(n, p):
    """The pivot reciprocals, read through the solve of a diagonal system
    with b = 1 (x_c is then the reciprocal of the pivot c): every component
    equals the exact rational 1/y rounded once, for pivots with parts close
    together, far apart, one part zero, powers of two and all-ones
    significands."""
    import torch
    import paper_2307_06072_amd as mp
    A = diagonal_pivots(n, p, [56, n, p])
    b = to_cmat(column([(Fraction(1), Fraction(0))] * n), p)
    _say(f"reciprocals n={n} p={p}")
    dA, ipiv, info = _factor(A, 16, p, 1)
    assert info == 0
    dB = mp.to_device(b)
    mp.mp_zgetrs(n, 1, dA, dA.ld, ipiv, dB, dB.ld, p, 1)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    X = device_result_to_host(dB, p)
    for c in range(n):
        R = lu_ref.reciprocal(lu_ref._sub(A, c, 1, c, 1), p)
        for name in ("re", "im"):
            got, want = getattr(X, name), getattr(R, name)
            assert int(got.exp[0, c]) == int(want.exp[0, 0]), (c, name)
            if int(want.exp[0, 0]) != -2 ** 31:
                assert int(got.sign[0, c]) == int(want.sign[0, 0]), (c, name)
                assert np.array_equal(got.mant[:, 0, c], want.mant[:, 0, 0]), (c, name)


def test_diagonal_shift_as_row_update():
    """The factorization workload's diagonal shift done on the device as the
    benchmark does it (the diagonal viewed as a 1 x n row with leading
    dimension lda + 1, plus n (1 + i) times a row of ones, one rounding)
    equals the host recipe bit for bit."""
    import torch
    import paper_2307_06072_amd as mp
    n, p = 128, 256  # n a power of two: n (1 + i) is written as 2^(e-1), e = bit length of n
    L = (p + 63) // 64
    A = random_cmat([5, n], 0, n, n, p, 2)
    want = dominant_matrix(n, p, [5, n])
    dA = mp.to_device(A)
    dn = mp.device_empty(1, 1, p)
    row1 = mp.device_empty(1, n, p)
    for part, e in ((dn.re, n.bit_length()), (dn.im, n.bit_length()), (row1.re, 1)):
        part.exp.fill_(e)
        part.mant[L - 1].fill_(-(1 << 63))
    diag = mp.DeviceCMat(1, n, dA.ld + 1, dA.L, dA.re, dA.im)
    mp.mpcg_set_stream()
    mp.mp_cgemm_acc(1, n, 1, dn, 1, row1, 1, diag, dA.ld + 1, p, +1)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    bad, first = mismatches(device_result_to_host(dA, p), want, n, n)
    assert bad == 0, (bad, first)


@pytest.mark.parametrize("nb", [4, 2])
def test_pivot_with_parts_90_bits_apart(nb):
    """Row 1 is row 0 plus 1 + 2^-90 i in column 1, and column 0's largest
    entries sit in rows 0 and 1, so elimination leaves the pivot 1 + 2^-90 i,
    whose parts are 90 bits apart although no entry of A has such a gap: the
    pivot search, the reciprocal and the scaling by it see the wide spread.
    Factors, interchanges and status equal the oracle's (U(1, 1) =
    1 + 2^-90 i exactly)."""
    import torch
    import paper_2307_06072_amd as mp
    F = Fraction
    p = 256
    e = F(2) ** -90
    vals = [[(F(8), F(0)), (F(1, 2), F(3, 4)), (F(3, 8), F(-1, 4)), (F(-1, 2), F(1, 8))],
            [(F(8), F(0)), (F(3, 2), F(3, 4) + e), (F(1, 4), F(1, 2)), (F(1, 8), F(-3, 8))],
            [(F(0), F(0)), (F(1, 4), F(1, 4)), (F(1), F(1, 2)), (F(1, 2), F(0))],
            [(F(0), F(0)), (F(-1, 4), F(1, 8)), (F(0), F(1, 2)), (F(1), F(-1, 4))]]
    A = to_cmat(vals, p)
    n = 4
    _say(f"getrf pivot 1 + 2^-90 i nb={nb}")
    dA, ipiv, info = _factor(A, nb, p, 1)
    ref, ref_piv, ref_info = lu_ref.getrf(A, nb, p)
    assert info == ref_info == 0
    assert np.array_equal(ipiv.cpu().numpy()[:n], ref_piv)
    F_dev = device_result_to_host(dA, p)
    bad, first = mismatches(F_dev, ref, n, n)
    assert bad == 0, (bad, first)
    assert decode(F_dev.im, 1, 1, p) == e
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
