"""Truncated scheme: the error bound against the oracle's unrounded exact value.

The bits of a truncated product are not unique (any value inside the bound is
correct), so these tests check the promised bound
    |C~ - C*| <= 2^-(p-4) * sum_k |a_ik|_max |b_kj|_max      (per component)
with C* the exact product from the oracle and |z|_max = max(|Re z|, |Im z|).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from mpgen import random_cmat, workload_inputs
from tests.gpu_util import run_device

pytestmark = pytest.mark.gpu

M4, M3 = 0, 1
EXACT, TRUNC = 0, 1
I8, F64 = 0, 1


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _absmax_terms(A, B, i, j):
    """sum_k |a_ik|_max |b_kj|_max as (numerator, exponent)."""
    terms = []
    for kk in range(A.cols):
        va = [oracle.entry_value(A.re, i, kk), oracle.entry_value(A.im, i, kk)]
        vb = [oracle.entry_value(B.re, kk, j), oracle.entry_value(B.im, kk, j)]
        a = _maxabs(va)
        b = _maxabs(vb)
        if a[0] == 0 or b[0] == 0:
            continue
        terms.append((a[0] * b[0], a[1] + b[1]))
    if not terms:
        return 0, 0
    e0 = min(e for _, e in terms)
    return sum(n << (e - e0) for n, e in terms), e0


def _maxabs(vals):
    best = (0, 0)
    for n, e in vals:
        n = abs(n)
        if n == 0:
            continue
        if best[0] == 0 or _cmp(n, e, best[0], best[1]) > 0:
            best = (n, e)
    return best


def _cmp(n1, e1, n2, e2):
    e = min(e1, e2)
    a, b = n1 << (e1 - e), n2 << (e2 - e)
    return (a > b) - (a < b)


def _bound_holds(got, exact, scale, p):
    """|got - exact| * 2^(p-4) <= scale, all (numerator, exponent) pairs, in integers."""
    (gn, ge), (xn, xe), (sn, se) = got, exact, scale
    e = min(ge, xe, se + 4 - p)
    diff = abs((gn << (ge - e)) - (xn << (xe - e)))
    rhs = sn << (se + 4 - p - e)
    return diff <= rhs, diff, rhs


def _check_bound(A, B, p, mode, slice_type, entries, **kw):
    _say(f"truncated m={A.rows} n={B.cols} k={A.cols} p={p} mode={mode} slice={slice_type} {kw}")
    C, info = run_device(A, B, p, mode, TRUNC, slice_type, **kw)
    assert info["bound_bits"] == p - 4
    worst = None
    for (i, j) in entries:
        scale = _absmax_terms(A, B, i, j)
        for comp, part in enumerate((C.re, C.im)):
            got = oracle.entry_value(part, i, j)
            exact = oracle.exact_entry(A, B, i, j, comp, p)
            ok, diff, rhs = _bound_holds(got, exact, scale, p)
            assert ok, (i, j, comp, info)
            if diff and rhs:
                r = diff.bit_length() - rhs.bit_length()
                worst = r if worst is None else max(worst, r)
    return info, worst


@pytest.mark.parametrize("mode,slice_type", [(M3, I8), (M4, I8), (M4, F64), (M3, F64)])
@pytest.mark.parametrize("R", [3, 40])
def test_truncated_bound_small(mode, slice_type, R):
    m, n, k, p = 18, 14, 45, 200
    A = random_cmat(40 + R, 0, m, k, p, R, zero_frac=0.1)
    B = random_cmat(40 + R, 1, k, n, p, R, zero_frac=0.1)
    entries = [(i, j) for i in range(m) for j in range(n)]
    info, _ = _check_bound(A, B, p, mode, slice_type, entries)
    _, exact_info = run_device(A, B, p, mode, EXACT, slice_type)
    assert info["pairs"] < exact_info["pairs"]


@pytest.mark.parametrize("p", [24, 64, 113, 640])
def test_truncated_bound_precisions(p):
    m, n, k = 12, 10, 33
    A = random_cmat(p + 7, 0, m, k, p, 6)
    B = random_cmat(p + 7, 1, k, n, p, 6)
    entries = [(i, j) for i in range(m) for j in range(n)]
    _check_bound(A, B, p, M3, I8, entries)
    _check_bound(A, B, p, M4, I8, entries)


def test_truncated_bound_cancellation():
    """Near-total cancellation: the bound is relative to sum |a||b|, not to |C|."""
    p, m, n, k = 128, 8, 8, 6
    A = random_cmat(77, 0, m, k, p, 4)
    B = random_cmat(77, 1, k, n, p, 4)
    for part in (A.re, A.im):  # column 1 = -column 0 (up to the last bit of the significand)
        part.exp[1] = part.exp[0]
        part.mant[:, 1] = part.mant[:, 0]
        part.mant[0, 1] ^= np.uint64(1) << np.uint64(64 - p % 64 if p % 64 else 0)
        part.sign[1] = part.sign[0] ^ 1
    for part in (B.re, B.im):
        part.exp[:, 1] = part.exp[:, 0]
        part.mant[:, :, 1] = part.mant[:, :, 0]
        part.sign[:, 1] = part.sign[:, 0]
    entries = [(i, j) for i in range(m) for j in range(n)]
    _check_bound(A, B, p, M3, I8, entries)
    _check_bound(A, B, p, M4, F64, entries)


def test_truncated_bound_config_512_p512_sampled():
    m, n, k, p, A, B = workload_inputs("cgemm512_p512")
    rng = np.random.default_rng(5)
    entries = list(zip(rng.integers(0, m, 40).tolist(), rng.integers(0, n, 40).tolist())) + [(0, 0), (m - 1, n - 1)]
    for mode, st in [(M3, I8), (M4, I8), (M4, F64)]:
        info, worst = _check_bound(A, B, p, mode, st, entries)
        _say(f"  pairs {info['pairs']} cutoff {info['cutoff']} worst log2(err/bound) {worst}")
