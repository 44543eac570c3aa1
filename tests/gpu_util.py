"""Helpers shared by the GPU tests: run the device path, compare with the oracle."""
from __future__ import annotations

import numpy as np

from mpgen import EXP_ZERO, HostCMat, HostPart


def device_result_to_host(C, prec_bits: int) -> HostCMat:
    import paper_2307_06072_amd as mp
    arr = mp.to_numpy(C)
    L = (prec_bits + 63) // 64
    parts = []
    for name in ("re", "im"):
        s, e, m = arr[name]
        parts.append(HostPart(C.rows, C.cols, C.ld, L, s, e, m))
    return HostCMat(*parts)


def run_device(A: HostCMat, B: HostCMat, prec_bits: int, mode: int, scheme: int, slice_type: int = 0, **kw):
    import torch
    import paper_2307_06072_amd as mp
    dA = mp.to_device(A)
    dB = mp.to_device(B)
    C, info = mp.matmul(dA, dB, prec_bits, mode=mode, scheme=scheme, slice_type=slice_type, **kw)
    torch.cuda.synchronize()
    st = mp.mpcg_stream_status()
    assert st == 0, f"device status {st}: {mp.mpcg_last_error()}"
    return device_result_to_host(C, prec_bits), info


def mismatches(C: HostCMat, R: HostCMat, m: int, n: int):
    """Component-wise bit comparison over the valid m x n block; zeros compare by exp only."""
    bad = 0
    first = None
    for name in ("re", "im"):
        c, r = getattr(C, name), getattr(R, name)
        ce, re_ = c.exp[:n, :m], r.exp[:n, :m]
        cz, rz = ce == EXP_ZERO, re_ == EXP_ZERO
        same = (ce == re_)
        nz = ~rz
        same &= np.where(nz, c.sign[:n, :m] == r.sign[:n, :m], True)
        same &= np.where(nz, np.all(c.mant[:, :n, :m] == r.mant[:, :n, :m], axis=0), True)
        same &= np.where(rz, cz, True)
        bad_here = ~same
        cnt = int(bad_here.sum())
        if cnt and first is None:
            j, i = np.argwhere(bad_here)[0]
            first = (name, int(i), int(j))
        bad += cnt
    return bad, first
