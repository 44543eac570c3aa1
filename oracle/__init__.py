"""CPU oracle for multi-precision complex matrix multiplication.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package imports nothing from the product path.

Two independent references live here:

* ``liboracle.so`` (``oracle_cgemm.c``): exact big-integer evaluation of
  C = AB (eq. 1/2 with the 4M expansion of eq. 3, or the 3M expansion of
  eq. 4), one round-to-nearest-even at the target precision per component.
* ``fraction_ref``: the same definition with ``fractions.Fraction`` and the
  textbook rounding rule, for tiny inputs only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from mpgen import EXP_ZERO, HostCMat, HostPart, empty_cmat

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_cgemm.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FORM_4M = 0
FORM_3M = 1


def build(extra_flags=()) -> str:
    """Compile liboracle.so with gcc (plain C, pthreads)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-fPIC", "-shared", "-pthread", *extra_flags,
           "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _InPart(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_void_p), ("exp", ctypes.c_void_p), ("mant", ctypes.c_void_p),
                ("limb_stride", ctypes.c_int64)]


class _InCMat(ctypes.Structure):
    _fields_ = [("re", _InPart), ("im", _InPart)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        override = os.environ.get("ORACLE_LIBRARY")  # another build, e.g. one with sanitizers
        if not override and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(override or _LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.oracle_cgemm.argtypes = [i32, i32, i32, vp, i64, vp, i64, vp, i64, i32, i32, i32]
        L.oracle_cgemm.restype = i32
        L.oracle_cgemm_entries.argtypes = [i32, i32, i32, vp, i64, vp, i64, i64, vp, vp, vp, vp, vp,
                                           i32, i32, i32]
        L.oracle_cgemm_entries.restype = i32
        L.oracle_exact_entry.argtypes = [i32, i32, i32, vp, i64, vp, i64, i32, i32, i32, i32, i32,
                                         vp, vp, vp, i32, vp]
        L.oracle_exact_entry.restype = i32
        L.oracle_cgemm_acc.argtypes = [i32, i32, i32, vp, i64, vp, i64, vp, i64, vp, i64, i32, i32, i32, i32]
        L.oracle_cgemm_acc.restype = i32
        L.oracle_cgemm_acc_entries.argtypes = [i32, i32, i32, vp, i64, vp, i64, vp, i64, i64, vp, vp, vp, vp,
                                               vp, i32, i32, i32, i32]
        L.oracle_cgemm_acc_entries.restype = i32
        _lib = L
    return _lib


class use_library:
    """Temporarily route this module's calls to another build of the oracle
    (used by the tests that plant mistakes in a copy of the source)."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib
        lib()
        self.saved = _lib
        L = ctypes.CDLL(self.path)
        for name in ("oracle_cgemm", "oracle_cgemm_entries", "oracle_exact_entry", "oracle_cgemm_acc",
                     "oracle_cgemm_acc_entries"):
            getattr(L, name).argtypes = getattr(self.saved, name).argtypes
            getattr(L, name).restype = getattr(self.saved, name).restype
        _lib = L
        return L

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _part_struct(p: HostPart, keep):
    for a in (p.sign, p.exp, p.mant):
        assert a.flags["C_CONTIGUOUS"]
        keep.append(a)
    return _InPart(p.sign.ctypes.data, p.exp.ctypes.data, p.mant.ctypes.data, p.cols * p.ld)


def _cmat_struct(M: HostCMat, keep):
    s = _InCMat(_part_struct(M.re, keep), _part_struct(M.im, keep))
    keep.append(s)
    return s


class OracleError(RuntimeError):
    pass


def _check(st: int, what: str):
    if st != 0:
        raise OracleError(f"{what}: oracle status {st}")


def cgemm(A: HostCMat, B: HostCMat, prec_bits: int, form: int = FORM_4M, nthreads: int | None = None,
          ldc: int | None = None) -> HostCMat:
    """Correctly rounded C = A B (every entry)."""
    m, k = A.rows, A.cols
    k2, n = B.rows, B.cols
    assert k == k2
    C = empty_cmat(m, n, prec_bits, ldc)
    keep = []
    a = _cmat_struct(A, keep)
    b = _cmat_struct(B, keep)
    c = _cmat_struct(C, keep)
    st = lib().oracle_cgemm(m, n, k, ctypes.addressof(a), A.ld, ctypes.addressof(b), B.ld,
                            ctypes.addressof(c), C.ld, prec_bits, form,
                            nthreads or default_threads())
    _check(st, "oracle_cgemm")
    return C


def cgemm_acc(A: HostCMat, B: HostCMat, Cin: HostCMat, prec_bits: int, sign: int = 1,
              form: int = FORM_4M, nthreads: int | None = None) -> HostCMat:
    """Correctly rounded C = Cin + sign * A B (every entry): the exact sum of the
    addend and the product, rounded once per component; sign is +1 or -1."""
    m, k = A.rows, A.cols
    n = B.cols
    assert B.rows == k and Cin.rows == m and Cin.cols == n
    C = empty_cmat(m, n, prec_bits)
    keep = []
    a = _cmat_struct(A, keep)
    b = _cmat_struct(B, keep)
    cin = _cmat_struct(Cin, keep)
    c = _cmat_struct(C, keep)
    st = lib().oracle_cgemm_acc(m, n, k, ctypes.addressof(a), A.ld, ctypes.addressof(b), B.ld,
                                ctypes.addressof(cin), Cin.ld, ctypes.addressof(c), C.ld, prec_bits, form,
                                sign, nthreads or default_threads())
    _check(st, "oracle_cgemm_acc")
    return C


def cgemm_acc_entries(A: HostCMat, B: HostCMat, Cin: HostCMat, rows, cols, prec_bits: int, sign: int = 1,
                      form: int = FORM_4M, nthreads: int | None = None):
    """Entries (rows[t], cols[t]) of the correctly rounded Cin + sign * A B, in
    the layout of cgemm_entries."""
    m, k = A.rows, A.cols
    n = B.cols
    ei = np.ascontiguousarray(rows, dtype=np.int32)
    ej = np.ascontiguousarray(cols, dtype=np.int32)
    nent = ei.size
    L = (prec_bits + 63) // 64
    sgn = np.zeros((nent, 2), np.uint8)
    exp = np.zeros((nent, 2), np.int32)
    mant = np.zeros((nent, 2, L), np.uint64)
    keep = []
    a = _cmat_struct(A, keep)
    b = _cmat_struct(B, keep)
    cin = _cmat_struct(Cin, keep)
    st = lib().oracle_cgemm_acc_entries(m, n, k, ctypes.addressof(a), A.ld, ctypes.addressof(b), B.ld,
                                        ctypes.addressof(cin), Cin.ld, nent, ei.ctypes.data, ej.ctypes.data,
                                        sgn.ctypes.data, exp.ctypes.data, mant.ctypes.data, prec_bits, form,
                                        sign, nthreads or default_threads())
    _check(st, "oracle_cgemm_acc_entries")
    return sgn, exp, mant


def cgemm_entries(A: HostCMat, B: HostCMat, rows, cols, prec_bits: int, form: int = FORM_4M,
                  nthreads: int | None = None):
    """Correctly rounded entries (rows[t], cols[t]).

    Returns (sign [nent, 2] uint8, exp [nent, 2] int32, mant [nent, 2, L] uint64),
    component 0 = Re, 1 = Im.
    """
    m, k = A.rows, A.cols
    n = B.cols
    ei = np.ascontiguousarray(rows, dtype=np.int32)
    ej = np.ascontiguousarray(cols, dtype=np.int32)
    nent = ei.size
    L = (prec_bits + 63) // 64
    sign = np.zeros((nent, 2), np.uint8)
    exp = np.zeros((nent, 2), np.int32)
    mant = np.zeros((nent, 2, L), np.uint64)
    keep = []
    a = _cmat_struct(A, keep)
    b = _cmat_struct(B, keep)
    st = lib().oracle_cgemm_entries(m, n, k, ctypes.addressof(a), A.ld, ctypes.addressof(b), B.ld,
                                    nent, ei.ctypes.data, ej.ctypes.data, sign.ctypes.data,
                                    exp.ctypes.data, mant.ctypes.data, prec_bits, form,
                                    nthreads or default_threads())
    _check(st, "oracle_cgemm_entries")
    return sign, exp, mant


def exact_entry(A: HostCMat, B: HostCMat, i: int, j: int, comp: int, prec_bits: int,
                form: int = FORM_4M):
    """Exact unrounded value of component ``comp`` of entry (i, j) as (numerator, exponent):
    value = numerator * 2**exponent, numerator a Python int (signed)."""
    m, k = A.rows, A.cols
    n = B.cols
    keep = []
    a = _cmat_struct(A, keep)
    b = _cmat_struct(B, keep)
    cap = 1 << 12
    while True:
        mag = np.zeros(cap, np.uint64)
        neg = ctypes.c_int(0)
        base = ctypes.c_int64(0)
        nmag = ctypes.c_int(0)
        st = lib().oracle_exact_entry(m, n, k, ctypes.addressof(a), A.ld, ctypes.addressof(b), B.ld,
                                      i, j, comp, prec_bits, form, ctypes.byref(neg),
                                      ctypes.byref(base), mag.ctypes.data, cap, ctypes.byref(nmag))
        if st == -2 and nmag.value > cap:
            cap = nmag.value
            continue
        _check(st, "oracle_exact_entry")
        break
    v = 0
    for t in range(nmag.value - 1, -1, -1):
        v = (v << 64) | int(mag[t])
    if neg.value:
        v = -v
    return v, int(base.value)


def entry_value(part: HostPart, idx_row: int, idx_col: int):
    """Decode one stored entry to (numerator, exponent) with value = num * 2**exponent."""
    e = int(part.exp[idx_col, idx_row])
    if e == EXP_ZERO:
        return 0, 0
    M = 0
    for l in range(part.L - 1, -1, -1):
        M = (M << 64) | int(part.mant[l, idx_col, idx_row])
    s = -1 if part.sign[idx_col, idx_row] else 1
    return s * M, e - 64 * part.L
