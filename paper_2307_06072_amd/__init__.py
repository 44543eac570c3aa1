"""Arbitrary-precision complex GEMM (Ozaki scheme, 4M/3M) on MI355X.

Thin ctypes binding over ``libmpcgemm.so``: the functions below carry the C
names of ``include/mpcgemm.h`` and only marshal arguments.  PyTorch supplies
device memory and the current stream; every step of the multiplication runs
in the library's HIP kernels.  There is no CPU fallback: importing this
package fails if the library has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MPCG_LIBRARY") or os.path.join(_HERE, "libmpcgemm.so")  # another build of the same sources

MPCG_OK = 0
MPCG_EINVAL = -1
MPCG_ENOMEM = -2
MPCG_ERANGE = -3
MPCG_EHIP = -4
MPCG_EUNSUPPORTED = -5
MPCG_EDOMAIN = -6
MPCG_ESPREAD = -7

MPCG_4M = 0
MPCG_3M = 1
MPCG_AUTO = 2
MPCG_EXACT = 0
MPCG_TRUNCATED = 1
MPCG_SLICE_INT8 = 0
MPCG_SLICE_FP64 = 1

EXP_ZERO = np.iinfo(np.int32).min

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python paper_2307_06072_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)


class mpcg_part(ctypes.Structure):
    _fields_ = [("sign", ctypes.c_void_p), ("exp", ctypes.c_void_p), ("mant", ctypes.c_void_p),
                ("limb_stride", ctypes.c_int64)]


class mpcg_cmat(ctypes.Structure):
    _fields_ = [("re", mpcg_part), ("im", mpcg_part)]


class mpcg_options(ctypes.Structure):
    _fields_ = [("slice_type", ctypes.c_int), ("cutoff_override", ctypes.c_int),
                ("ksplit_override", ctypes.c_int), ("block_override", ctypes.c_int),
                ("max_spread", ctypes.c_int), ("adaptive", ctypes.c_int), ("strassen", ctypes.c_int),
                ("part_scales", ctypes.c_int)]


class mpcg_info(ctypes.Structure):
    _fields_ = [("S_A", ctypes.c_int), ("S_B", ctypes.c_int), ("w", ctypes.c_int), ("cutoff", ctypes.c_int),
                ("nprod", ctypes.c_int), ("ksplit", ctypes.c_int), ("block", ctypes.c_int),
                ("strassen", ctypes.c_int), ("pairs", ctypes.c_longlong), ("algo_ops", ctypes.c_double),
                ("bound_bits", ctypes.c_double), ("part_scales", ctypes.c_int), ("apart", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mpcg_tune_report(ctypes.Structure):
    _fields_ = [("band", ctypes.c_int), ("groups", ctypes.c_int), ("mode", ctypes.c_int), ("S", ctypes.c_int),
                ("candidates", ctypes.c_int), ("us", ctypes.c_float), ("untuned_us", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class mpcg_problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("k", ctypes.c_int),
                ("A", ctypes.POINTER(mpcg_cmat)), ("lda", ctypes.c_int),
                ("B", ctypes.POINTER(mpcg_cmat)), ("ldb", ctypes.c_int),
                ("C", ctypes.POINTER(mpcg_cmat)), ("ldc", ctypes.c_int)]


_P = ctypes.POINTER
_i = ctypes.c_int
_vp = ctypes.c_void_p
_lib.mp_cgemm.argtypes = [_i, _i, _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _i, _i, _i]
_lib.mp_cgemm.restype = _i
_lib.mp_cgemm_ex.argtypes = [_i, _i, _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _i, _i, _i,
                             _P(mpcg_options), _P(mpcg_info)]
_lib.mp_cgemm_ex.restype = _i
_lib.mp_cgemm_ex_noalloc.argtypes = [_i, _i, _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _i, _i,
                                     _i, _P(mpcg_options), _P(mpcg_info)]
_lib.mp_cgemm_ex_noalloc.restype = _i
_lib.mp_cgemm_acc.argtypes = [_i, _i, _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _i, _i, _i, _i,
                              _P(mpcg_options), _P(mpcg_info)]
_lib.mp_cgemm_acc.restype = _i
_lib.mp_cgemm_batched.argtypes = [_i, _P(mpcg_problem), _i, _i, _i, _P(mpcg_options), _P(mpcg_info)]
_lib.mp_cgemm_batched.restype = _i
_lib.mp_cgemm_batched_acc.argtypes = [_i, _P(mpcg_problem), _i, _i, _i, _i, _P(mpcg_options), _P(mpcg_info)]
_lib.mp_cgemm_batched_acc.restype = _i
_lib.mpcg_set_stream.argtypes = [_vp]
_lib.mpcg_set_stream.restype = _i
_lib.mpcg_set_workspace.argtypes = [_vp, ctypes.c_size_t]
_lib.mpcg_set_workspace.restype = _i
_lib.mpcg_workspace_size.argtypes = [_i, _i, _i, _i, _i, _i, _P(mpcg_options), _i]
_lib.mpcg_workspace_size.restype = ctypes.c_size_t
_lib.mpcg_workspace_size_batched.argtypes = [_i, _P(mpcg_problem), _i, _i, _i, _P(mpcg_options)]
_lib.mpcg_workspace_size_batched.restype = ctypes.c_size_t
_lib.mpcg_autotune.argtypes = [_i, _i, _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _P(mpcg_cmat), _i, _i, _i, _i, _i,
                               _P(mpcg_tune_report)]
_lib.mpcg_autotune.restype = _i
_lib.mpcg_autotune_batched.argtypes = [_i, _P(mpcg_problem), _i, _i, _i, _i, _P(mpcg_options), _P(mpcg_tune_report)]
_lib.mpcg_autotune_batched.restype = _i
_lib.mpcg_tune_load.argtypes = [ctypes.c_char_p]
_lib.mpcg_tune_load.restype = _i
_lib.mpcg_tune_save.argtypes = [ctypes.c_char_p]
_lib.mpcg_tune_save.restype = _i
_lib.mpcg_tune_clear.argtypes = []
_lib.mpcg_tune_clear.restype = _i
_lib.mpcg_stream_status.argtypes = [_vp]
_lib.mpcg_stream_status.restype = _i
_lib.mpcg_last_error.argtypes = []
_lib.mpcg_last_error.restype = ctypes.c_char_p
_lib.mpcg_enable_timing.argtypes = [_i]
_lib.mpcg_enable_timing.restype = _i
_lib.mpcg_last_timing.argtypes = [_P(ctypes.c_float)]
_lib.mpcg_last_timing.restype = _i
_lib.mpcg_timing_report.argtypes = [_P(ctypes.c_float), _P(ctypes.c_int)]
_lib.mpcg_timing_report.restype = _i
_lib.mpcg_probe_mfma.argtypes = [_i, _i, _i, _vp, _P(ctypes.c_double), _P(ctypes.c_float)]
_lib.mpcg_probe_mfma.restype = _i
_lib.mpcg_from_doubles.argtypes = [_i, _i, _i, _vp, _i, ctypes.c_longlong, _P(mpcg_part), _i, _i]
_lib.mpcg_from_doubles.restype = _i
_lib.mpcg_to_doubles.argtypes = [_i, _i, _P(mpcg_part), _i, _i, _i, _vp, _i, ctypes.c_longlong]
_lib.mpcg_to_doubles.restype = _i
_lib.mp_zgetrf.argtypes = [_i, _P(mpcg_cmat), _i, _vp, _i, _i, _i]
_lib.mp_zgetrf.restype = _i
_lib.mp_zgetrs.argtypes = [_i, _i, _P(mpcg_cmat), _i, _vp, _P(mpcg_cmat), _i, _i, _i]
_lib.mp_zgetrs.restype = _i

EXPORTS = ["mp_cgemm", "mp_cgemm_ex", "mp_cgemm_ex_noalloc", "mp_cgemm_acc", "mp_cgemm_batched", "mp_cgemm_batched_acc", "mp_zgetrf", "mp_zgetrs", "mpcg_set_stream", "mpcg_set_workspace", "mpcg_workspace_size", "mpcg_workspace_size_batched", "mpcg_autotune", "mpcg_autotune_batched", "mpcg_tune_load",
           "mpcg_tune_save", "mpcg_tune_clear",
           "mpcg_stream_status", "mpcg_last_error", "mpcg_enable_timing", "mpcg_last_timing",
           "mpcg_timing_report", "mpcg_from_doubles", "mpcg_to_doubles", "mpcg_probe_mfma"]


class MPCGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mpcgemm error {code}: {msg}")
        self.code = code


def mpcg_last_error() -> str:
    return (_lib.mpcg_last_error() or b"").decode()


def _check(code: int) -> int:
    if code != MPCG_OK:
        raise MPCGError(code, mpcg_last_error())
    return code


# ---------------------------------------------------------------------------
# Device matrices: torch tensors used as plain device memory.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DevicePart:
    sign: "object"  # torch.uint8 [cols, ld]
    exp: "object"   # torch.int32 [cols, ld]
    mant: "object"  # torch.int64 [L, cols, ld] (uint64 bit patterns)

    def struct(self) -> mpcg_part:
        return mpcg_part(self.sign.data_ptr(), self.exp.data_ptr(), self.mant.data_ptr(),
                         self.mant.shape[1] * self.mant.shape[2])


@dataclasses.dataclass
class DeviceCMat:
    rows: int
    cols: int
    ld: int
    L: int
    re: DevicePart
    im: DevicePart

    def struct(self) -> mpcg_cmat:
        return mpcg_cmat(self.re.struct(), self.im.struct())


def _torch():
    import torch
    return torch


def device_empty(rows: int, cols: int, prec_bits: int, ld: int | None = None, device="cuda") -> DeviceCMat:
    torch = _torch()
    ld = max(1, rows) if ld is None else ld
    L = (prec_bits + 63) // 64

    def part():
        return DevicePart(torch.zeros((cols, ld), dtype=torch.uint8, device=device),
                          torch.full((cols, ld), EXP_ZERO, dtype=torch.int32, device=device),
                          torch.zeros((L, cols, ld), dtype=torch.int64, device=device))
    return DeviceCMat(rows, cols, ld, L, part(), part())


def to_device(host, device="cuda") -> DeviceCMat:
    """Upload a host matrix (objects with .re/.im parts holding sign/exp/mant numpy arrays)."""
    torch = _torch()

    def part(p):
        return DevicePart(torch.from_numpy(np.ascontiguousarray(p.sign)).to(device),
                          torch.from_numpy(np.ascontiguousarray(p.exp)).to(device),
                          torch.from_numpy(np.ascontiguousarray(p.mant).view(np.int64)).to(device))
    # an empty matrix still has a leading dimension of at least 1 (BLAS convention)
    return DeviceCMat(host.rows, host.cols, max(1, host.ld), host.L, part(host.re), part(host.im))


def to_numpy(dev: DeviceCMat):
    """Download: returns dict of numpy arrays {re: (sign, exp, mant), im: (...)} (mant as uint64)."""
    out = {}
    for name in ("re", "im"):
        p = getattr(dev, name)
        out[name] = (p.sign.cpu().numpy(), p.exp.cpu().numpy(), p.mant.cpu().numpy().view(np.uint64))
    return out


def current_stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# C entry points (same names as the header).
# ---------------------------------------------------------------------------
def mpcg_set_stream(stream=None) -> int:
    """Bind the library to a HIP stream (default: torch's current stream)."""
    if stream is None:
        stream = current_stream_handle()
    elif not isinstance(stream, ctypes.c_void_p):
        stream = ctypes.c_void_p(int(stream))
    return _check(_lib.mpcg_set_stream(stream))


def mpcg_set_workspace(ptr: int | None, nbytes: int) -> int:
    return _check(_lib.mpcg_set_workspace(ctypes.c_void_p(ptr) if ptr else None, nbytes))


def mpcg_workspace_size(m, n, k, prec_bits, mode=MPCG_3M, scheme=MPCG_EXACT, options=None,
                        max_spread=0) -> int:
    opt = ctypes.byref(options) if options is not None else None
    return int(_lib.mpcg_workspace_size(m, n, k, prec_bits, mode, scheme, opt, max_spread))


def mpcg_stream_status(stream=None) -> int:
    if stream is None:
        stream = current_stream_handle()
    return int(_lib.mpcg_stream_status(stream))


def mpcg_from_doubles(rows, cols, ncomp, src_ptr, ld, plane, dst: DevicePart, ldd, prec_bits) -> int:
    return int(_lib.mpcg_from_doubles(rows, cols, ncomp, src_ptr, ld, plane, ctypes.byref(dst.struct()), ldd,
                                      prec_bits))


def from_doubles(re, im, prec_bits: int) -> DeviceCMat:
    """Multi-component inputs: re and im are float64 device tensors of shape
    (ncomp, cols, rows) (component planes, column-major entries); entry
    (r, c) of each part is the exact sum of its ncomp doubles.  Returns the
    complex matrix in the library's format at prec_bits, each sum rounded
    once (mpcg_from_doubles, on the library's stream)."""
    torch = _torch()
    ncomp, cols, rows = re.shape
    if im.shape != re.shape or re.dtype != torch.float64 or im.dtype != torch.float64:
        raise ValueError("re and im must be float64 tensors of the same shape (ncomp, cols, rows)")
    re, im = re.contiguous(), im.contiguous()
    C = device_empty(rows, cols, prec_bits, device=re.device)
    for t, part in ((re, C.re), (im, C.im)):
        _check(mpcg_from_doubles(rows, cols, ncomp, t.data_ptr(), max(1, rows), max(1, rows) * cols, part,
                                     C.ld, prec_bits))
    return C


def mpcg_to_doubles(rows, cols, src: DevicePart, lds, prec_bits, ncomp, dst_ptr, ld, plane) -> int:
    return int(_lib.mpcg_to_doubles(rows, cols, ctypes.byref(src.struct()), lds, prec_bits, ncomp, dst_ptr, ld,
                                    plane))


def to_doubles(C: DeviceCMat, prec_bits: int, ncomp: int):
    """The opposite of from_doubles: (re, im) float64 device tensors of shape
    (ncomp, cols, rows), each entry's components chosen greedily (each the
    double nearest what the earlier ones leave; mpcg_to_doubles)."""
    torch = _torch()
    out = []
    for part in (C.re, C.im):
        t = torch.empty((ncomp, C.cols, max(1, C.rows)), dtype=torch.float64, device=part.exp.device)
        _check(mpcg_to_doubles(C.rows, C.cols, part, C.ld, prec_bits, ncomp, t.data_ptr(), max(1, C.rows),
                               max(1, C.rows) * C.cols))
        out.append(t)
    return tuple(out)


def mpcg_enable_timing(on: bool = True) -> int:
    return _check(_lib.mpcg_enable_timing(1 if on else 0))


def mpcg_last_timing():
    us = (ctypes.c_float * 4)()
    _check(_lib.mpcg_last_timing(us))
    return list(us)


def mpcg_probe_mfma(kind: int, blocks: int, iters: int, sink_ptr: int):
    """Matrix-core rate probe (kind 0: INT8 16x16x64, 1: FP64 16x16x4):
    (operations issued, kernel milliseconds).  sink_ptr: a device buffer of
    at least 4 bytes."""
    ops = ctypes.c_double(0.0)
    ms = ctypes.c_float(0.0)
    _check(_lib.mpcg_probe_mfma(kind, blocks, iters, ctypes.c_void_p(sink_ptr), ctypes.byref(ops), ctypes.byref(ms)))
    return ops.value, ms.value


def mpcg_timing_report():
    """(per-stage microseconds summed over the recorded calls, number of calls)."""
    us = (ctypes.c_float * 4)()
    n = ctypes.c_int(0)
    _check(_lib.mpcg_timing_report(us, ctypes.byref(n)))
    return list(us), n.value


def mp_cgemm_raw(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme) -> int:
    """Direct call with ctypes structs/pointers (or None); returns the status code unchanged."""
    return int(_lib.mp_cgemm(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme))


def mp_cgemm_ex_raw(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, options=None, info=None) -> int:
    return int(_lib.mp_cgemm_ex(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, options, info))


def mp_cgemm(m, n, k, A: DeviceCMat, lda, B: DeviceCMat, ldb, C: DeviceCMat, ldc, prec_bits,
             mode=MPCG_3M, scheme=MPCG_EXACT) -> int:
    a, b, c = A.struct(), B.struct(), C.struct()
    return _check(_lib.mp_cgemm(m, n, k, ctypes.byref(a), lda, ctypes.byref(b), ldb, ctypes.byref(c), ldc,
                                prec_bits, mode, scheme))


def mp_cgemm_ex(m, n, k, A: DeviceCMat, lda, B: DeviceCMat, ldb, C: DeviceCMat, ldc, prec_bits,
                mode=MPCG_3M, scheme=MPCG_EXACT, slice_type=MPCG_SLICE_INT8, cutoff_override=0,
                ksplit_override=0, block_override=0, max_spread=0, adaptive=0, strassen=0, part_scales=0) -> dict:
    a, b, c = A.struct(), B.struct(), C.struct()
    opt = mpcg_options(slice_type, cutoff_override, ksplit_override, block_override, max_spread, adaptive, strassen,
                       part_scales)
    info = mpcg_info()
    _check(_lib.mp_cgemm_ex(m, n, k, ctypes.byref(a), lda, ctypes.byref(b), ldb, ctypes.byref(c), ldc,
                            prec_bits, mode, scheme, ctypes.byref(opt), ctypes.byref(info)))
    return info.as_dict()


def mp_cgemm_ex_noalloc_raw(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, options=None,
                            info=None) -> int:
    return int(_lib.mp_cgemm_ex_noalloc(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, options, info))


def mp_cgemm_ex_noalloc(m, n, k, A: DeviceCMat, lda, B: DeviceCMat, ldb, C: DeviceCMat, ldc, prec_bits,
                        mode=MPCG_3M, scheme=MPCG_EXACT, slice_type=MPCG_SLICE_INT8, cutoff_override=0,
                        ksplit_override=0, block_override=0, max_spread=0) -> dict:
    """mp_cgemm_ex with every scratch byte from the library's fixed device
    buffer (MPCG_NOALLOC_BYTES per device); no allocation."""
    a, b, c = A.struct(), B.struct(), C.struct()
    opt = mpcg_options(slice_type, cutoff_override, ksplit_override, block_override, max_spread, 0)
    info = mpcg_info()
    _check(_lib.mp_cgemm_ex_noalloc(m, n, k, ctypes.byref(a), lda, ctypes.byref(b), ldb, ctypes.byref(c), ldc,
                                    prec_bits, mode, scheme, ctypes.byref(opt), ctypes.byref(info)))
    return info.as_dict()


def mpcg_autotune(m, n, k, A: DeviceCMat, lda, B: DeviceCMat, ldb, C: DeviceCMat, ldc, prec_bits, mode=MPCG_AUTO,
                  scheme=MPCG_EXACT, reps=2) -> dict:
    """Measure the plans of this product and store the fastest for its size
    class; returns the choice (band, groups, mode, S, candidates, us,
    untuned_us).  C is overwritten."""
    a, b, c = A.struct(), B.struct(), C.struct()
    rep = mpcg_tune_report()
    _check(_lib.mpcg_autotune(m, n, k, ctypes.byref(a), lda, ctypes.byref(b), ldb, ctypes.byref(c), ldc, prec_bits,
                              mode, scheme, reps, ctypes.byref(rep)))
    return rep.as_dict()


def mpcg_autotune_batched(problems, prec_bits, mode=MPCG_AUTO, scheme=MPCG_EXACT, reps=1, max_spread=0) -> dict:
    """Tune a batch of (A, B, C) triples: one band width and form for the whole
    batch if that beats each problem's own; stored per size class."""
    arr, keep = _problem_array(problems)
    opt = mpcg_options(MPCG_SLICE_INT8, 0, 0, 0, max_spread)
    rep = mpcg_tune_report()
    _check(_lib.mpcg_autotune_batched(len(problems), arr, prec_bits, mode, scheme, reps, ctypes.byref(opt),
                                      ctypes.byref(rep)))
    return rep.as_dict()


def _count(code: int) -> int:
    if code < 0:
        raise MPCGError(code, mpcg_last_error())
    return code


def mpcg_tune_load(path=None) -> int:
    """Merge a tuning cache file (None: $MPCG_TUNE_CACHE); returns entries read."""
    return _count(_lib.mpcg_tune_load(path.encode() if path else None))


def mpcg_tune_save(path=None) -> int:
    """Write the tuning cache (None: $MPCG_TUNE_CACHE); returns entries written."""
    return _count(_lib.mpcg_tune_save(path.encode() if path else None))


def mpcg_tune_clear() -> int:
    return _check(_lib.mpcg_tune_clear())


def mp_cgemm_acc_raw(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, sign, options=None,
                     info=None) -> int:
    return int(_lib.mp_cgemm_acc(m, n, k, A, lda, B, ldb, C, ldc, prec_bits, mode, scheme, sign, options, info))


def mp_cgemm_acc(m, n, k, A: DeviceCMat, lda, B: DeviceCMat, ldb, C: DeviceCMat, ldc, prec_bits, sign=-1,
                 mode=MPCG_3M, scheme=MPCG_EXACT, cutoff_override=0, ksplit_override=0, block_override=0,
                 max_spread=0, adaptive=0) -> dict:
    """C := C + sign * A B in place (sign = +1 or -1), one rounding."""
    a, b, c = A.struct(), B.struct(), C.struct()
    opt = mpcg_options(MPCG_SLICE_INT8, cutoff_override, ksplit_override, block_override, max_spread, adaptive)
    info = mpcg_info()
    _check(_lib.mp_cgemm_acc(m, n, k, ctypes.byref(a), lda, ctypes.byref(b), ldb, ctypes.byref(c), ldc,
                             prec_bits, mode, scheme, sign, ctypes.byref(opt), ctypes.byref(info)))
    return info.as_dict()


def mp_cgemm_batched_raw(count, problems, prec_bits, mode, scheme, options=None, info=None) -> int:
    return int(_lib.mp_cgemm_batched(count, problems, prec_bits, mode, scheme, options, info))


def _problem_array(problems):
    keep = []
    arr = (mpcg_problem * max(1, len(problems)))()
    for t, (A, B, C) in enumerate(problems):
        a, b, c = A.struct(), B.struct(), C.struct()
        keep += [a, b, c]
        arr[t] = mpcg_problem(A.rows, B.cols, A.cols, ctypes.pointer(a), A.ld, ctypes.pointer(b), B.ld,
                              ctypes.pointer(c), C.ld)
    return arr, keep


def mpcg_workspace_size_batched(problems, prec_bits, mode=MPCG_3M, scheme=MPCG_EXACT, max_spread=0,
                                block_override=0, ksplit_override=0) -> int:
    """Workspace bytes of a batch planned from max_spread (> 0)."""
    arr, keep = _problem_array(problems)
    opt = mpcg_options(MPCG_SLICE_INT8, 0, ksplit_override, block_override, max_spread)
    return int(_lib.mpcg_workspace_size_batched(len(problems), arr, prec_bits, mode, scheme, ctypes.byref(opt)))


def mp_cgemm_batched(problems, prec_bits, mode=MPCG_3M, scheme=MPCG_EXACT, cutoff_override=0,
                     ksplit_override=0, block_override=0, max_spread=0) -> dict:
    """problems: sequence of (A, B, C) DeviceCMat triples (C := A B each, leading
    dimensions from the matrices).  Returns the summed plan report."""
    keep = []
    arr = (mpcg_problem * max(1, len(problems)))()
    for t, (A, B, C) in enumerate(problems):
        a, b, c = A.struct(), B.struct(), C.struct()
        keep += [a, b, c]
        arr[t] = mpcg_problem(A.rows, B.cols, A.cols, ctypes.pointer(a), A.ld, ctypes.pointer(b), B.ld,
                              ctypes.pointer(c), C.ld)
    opt = mpcg_options(MPCG_SLICE_INT8, cutoff_override, ksplit_override, block_override, max_spread)
    info = mpcg_info()
    _check(_lib.mp_cgemm_batched(len(problems), arr, prec_bits, mode, scheme, ctypes.byref(opt),
                                 ctypes.byref(info)))
    return info.as_dict()


def mp_cgemm_batched_acc_raw(count, problems, prec_bits, mode, scheme, sign, options=None, info=None) -> int:
    return int(_lib.mp_cgemm_batched_acc(count, problems, prec_bits, mode, scheme, sign, options, info))


def mp_cgemm_batched_acc(problems, prec_bits, sign=-1, mode=MPCG_3M, scheme=MPCG_EXACT, cutoff_override=0,
                         ksplit_override=0, block_override=0, max_spread=0) -> dict:
    """problems: sequence of (A, B, C) DeviceCMat triples; C := C + sign * A B
    in place for each.  Returns the summed plan report."""
    keep = []
    arr = (mpcg_problem * max(1, len(problems)))()
    for t, (A, B, C) in enumerate(problems):
        a, b, c = A.struct(), B.struct(), C.struct()
        keep += [a, b, c]
        arr[t] = mpcg_problem(A.rows, B.cols, A.cols, ctypes.pointer(a), A.ld, ctypes.pointer(b), B.ld,
                              ctypes.pointer(c), C.ld)
    opt = mpcg_options(MPCG_SLICE_INT8, cutoff_override, ksplit_override, block_override, max_spread)
    info = mpcg_info()
    _check(_lib.mp_cgemm_batched_acc(len(problems), arr, prec_bits, mode, scheme, sign, ctypes.byref(opt),
                                     ctypes.byref(info)))
    return info.as_dict()


def mp_zgetrf_raw(n, A, lda, ipiv_ptr, nb, prec_bits, mode) -> int:
    return int(_lib.mp_zgetrf(n, A, lda, ipiv_ptr, nb, prec_bits, mode))


def mp_zgetrf(n, A: DeviceCMat, lda, ipiv, nb, prec_bits, mode=MPCG_3M) -> int:
    """Blocked LU with partial pivoting in place; ipiv is an int32 device
    tensor of n entries (0-based interchanges).  Returns 0 or c + 1 for the
    first zero pivot in column c (negative codes raise)."""
    a = A.struct()
    st = int(_lib.mp_zgetrf(n, ctypes.byref(a), lda, ipiv.data_ptr() if n else None, nb, prec_bits, mode))
    return st if st > 0 else _check(st)


def mp_zgetrs_raw(n, nrhs, A, lda, ipiv_ptr, B, ldb, prec_bits, mode) -> int:
    return int(_lib.mp_zgetrs(n, nrhs, A, lda, ipiv_ptr, B, ldb, prec_bits, mode))


def mp_zgetrs(n, nrhs, A: DeviceCMat, lda, ipiv, B: DeviceCMat, ldb, prec_bits, mode=MPCG_3M) -> int:
    """Solve A X = B with the factors of mp_zgetrf; B is overwritten by X."""
    a, b = A.struct(), B.struct()
    return _check(_lib.mp_zgetrs(n, nrhs, ctypes.byref(a), lda, ipiv.data_ptr() if n else None, ctypes.byref(b),
                                 ldb, prec_bits, mode))


def matmul(A: DeviceCMat, B: DeviceCMat, prec_bits: int, mode=MPCG_3M, scheme=MPCG_EXACT,
           slice_type=MPCG_SLICE_INT8, **kw):
    """Convenience: allocate C and run mp_cgemm_ex on torch's current stream. Returns (C, info)."""
    C = device_empty(A.rows, B.cols, prec_bits, device=A.re.sign.device)
    mpcg_set_stream()
    info = mp_cgemm_ex(A.rows, B.cols, A.cols, A, A.ld, B, B.ld, C, C.ld, prec_bits, mode, scheme,
                       slice_type=slice_type, **kw)
    return C, info
