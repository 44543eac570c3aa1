"""C-ABI library: loads, exports every declared symbol, and validates
arguments on the host before any device work (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcgemm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for must in ("mp_cgemm", "mp_cgemm_ex", "mpcg_set_stream", "mpcg_set_workspace",
                 "mpcg_workspace_size", "mpcg_stream_status", "mpcg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2307_06072_amd as mp
    lib = ctypes.CDLL(mp.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_has_same_names():
    import paper_2307_06072_amd as mp
    for n in _declared_functions():
        assert hasattr(mp, n), n


# ---------------------------------------------------------------------------
# validation runs on the host, before any HIP call
# ---------------------------------------------------------------------------
def _fake_cmat(base: int):
    import paper_2307_06072_amd as mp
    # distinct fake device addresses, far apart; never dereferenced on the host
    def part(off):
        return mp.mpcg_part(base + off, base + off + (1 << 24), base + off + (2 << 24), 0)
    return mp.mpcg_cmat(part(0), part(3 << 24))


def _call(m=4, n=4, k=4, lda=4, ldb=4, ldc=4, p=256, mode=1, scheme=0, A=None, B=None, C=None, opt=None):
    import paper_2307_06072_amd as mp
    A = _fake_cmat(1 << 40) if A is None else A
    B = _fake_cmat(2 << 40) if B is None else B
    C = _fake_cmat(3 << 40) if C is None else C
    pa = ctypes.byref(A) if A is not False else None
    pb = ctypes.byref(B) if B is not False else None
    pc = ctypes.byref(C) if C is not False else None
    if opt is not None:
        return mp.mp_cgemm_ex_raw(m, n, k, pa, lda, pb, ldb, pc, ldc, p, mode, scheme, ctypes.byref(opt), None)
    return mp.mp_cgemm_raw(m, n, k, pa, lda, pb, ldb, pc, ldc, p, mode, scheme)


@pytest.mark.parametrize("kw", [dict(m=-1), dict(n=-2), dict(k=-3), dict(lda=3), dict(ldb=3), dict(ldc=2),
                                dict(p=1), dict(p=4097), dict(mode=3), dict(scheme=5), dict(A=False),
                                dict(B=False), dict(C=False)])
def test_invalid_arguments(kw):
    import paper_2307_06072_amd as mp
    assert _call(**kw) == mp.MPCG_EINVAL
    assert mp.mpcg_last_error() != ""


def test_null_component_pointer():
    import paper_2307_06072_amd as mp
    A = _fake_cmat(1 << 40)
    A.im.mant = None
    assert _call(A=A) == mp.MPCG_EINVAL
    assert "NULL" in mp.mpcg_last_error()


def test_limb_stride_too_small():
    import paper_2307_06072_amd as mp
    B = _fake_cmat(2 << 40)
    B.re.limb_stride = 15  # ld*cols = 16
    assert _call(B=B) == mp.MPCG_EINVAL


def test_limb_stride_covers_only_the_addressed_entries():
    """A strided row view (the diagonal of a 4 x 4 matrix as a 1 x 4 row with
    ld = 5) addresses entries 0, 5, 10, 15: a limb stride of 16 keeps the limb
    planes apart and passes validation (the call then fails only at its
    first device call on a host without a GPU); 15 is rejected."""
    import paper_2307_06072_amd as mp
    for ls, bad in ((16, False), (15, True)):
        C = _fake_cmat(3 << 40)
        C.re.limb_stride = ls
        C.im.limb_stride = ls
        rc = _call(m=1, n=4, k=4, ldc=5, C=C)
        assert (rc == mp.MPCG_EINVAL) == bad, (ls, rc, mp.mpcg_last_error())


def test_output_aliasing_input_rejected():
    import paper_2307_06072_amd as mp
    A = _fake_cmat(1 << 40)
    C = _fake_cmat(3 << 40)
    C.im.exp = A.re.exp + 8  # overlaps A's exponent array
    assert _call(A=A, C=C) == mp.MPCG_EINVAL
    assert "overlap" in mp.mpcg_last_error()


def test_bad_options_rejected():
    import paper_2307_06072_amd as mp
    assert _call(opt=mp.mpcg_options(7, 0, 0, 0)) == mp.MPCG_EINVAL
    assert _call(opt=mp.mpcg_options(0, -1, 0, 0)) == mp.MPCG_EINVAL


def test_quick_return_empty_output():
    # m == 0 or n == 0: nothing to do, even with NULL matrices
    assert _call(m=0, A=False, B=False, C=False) == 0
    assert _call(n=0, A=False, B=False, C=False) == 0


def test_workspace_size_planning():
    import paper_2307_06072_amd as mp
    s1 = mp.mpcg_workspace_size(512, 512, 512, 512, mp.MPCG_3M, mp.MPCG_EXACT, None, 16)
    s2 = mp.mpcg_workspace_size(512, 512, 512, 512, mp.MPCG_3M, mp.MPCG_TRUNCATED, None, 16)
    s3 = mp.mpcg_workspace_size(512, 512, 512, 1024, mp.MPCG_3M, mp.MPCG_EXACT, None, 16)
    assert 0 < s2 < s1 < s3
    assert mp.mpcg_workspace_size(0, 5, 5, 256) == 0


def test_injected_hip_failure_is_reported():
    """MPCG_FAULT_INJECT=hip makes the first HIP call fail: the status is MPCG_EHIP."""
    code = (
        "import ctypes, sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from tests.test_abi import _call\n"
        "import paper_2307_06072_amd as mp\n"
        "rc = _call(k=0)\n"
        "print(rc, mp.mpcg_last_error())\n"
        "sys.exit(0 if rc == mp.MPCG_EHIP else 1)\n")
    env = dict(os.environ, MPCG_FAULT_INJECT="hip", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr


# ---------------------------------------------------------------------------
# batched entry point: validation before any device work
# ---------------------------------------------------------------------------
def _batch_call(probs, p=256, mode=1, scheme=0, opt=None, count=None):
    import paper_2307_06072_amd as mp
    keep = []
    arr = (mp.mpcg_problem * max(1, len(probs)))()
    for t, (m, n, k, A, B, C, lda, ldb, ldc) in enumerate(probs):
        keep += [A, B, C]
        arr[t] = mp.mpcg_problem(m, n, k, ctypes.pointer(A) if A is not None else None, lda,
                                 ctypes.pointer(B) if B is not None else None, ldb,
                                 ctypes.pointer(C) if C is not None else None, ldc)
    o = ctypes.byref(opt) if opt is not None else None
    return mp.mp_cgemm_batched_raw(len(probs) if count is None else count, arr, p, mode, scheme, o, None)


def _prob(t, m=4, n=4, k=4):
    return (m, n, k, _fake_cmat((1 + 3 * t) << 40), _fake_cmat((2 + 3 * t) << 40), _fake_cmat((3 + 3 * t) << 40),
            max(1, m), max(1, k), max(1, m))


def test_batched_validation():
    import paper_2307_06072_amd as mp
    assert _batch_call([], count=0) == mp.MPCG_OK
    assert _batch_call([_prob(0)], count=-1) == mp.MPCG_EINVAL
    assert mp.mp_cgemm_batched_raw(2, None, 256, 1, 0, None, None) == mp.MPCG_EINVAL
    bad = list(_prob(1))
    bad[6] = 2  # lda < m
    assert _batch_call([_prob(0), tuple(bad)]) == mp.MPCG_EINVAL
    assert "problem 1" in mp.mpcg_last_error()
    assert _batch_call([_prob(0)], p=1) == mp.MPCG_EINVAL
    assert _batch_call([_prob(0)], mode=3) == mp.MPCG_EINVAL
    assert _batch_call([_prob(0)], opt=mp.mpcg_options(1, 0, 0, 0, 0)) == mp.MPCG_EUNSUPPORTED
    assert _batch_call([_prob(0)], opt=mp.mpcg_options(0, 0, 0, 0, -4)) == mp.MPCG_EINVAL
    # nothing to compute: empty outputs need no device
    assert _batch_call([_prob(0, m=0), _prob(1, n=0)]) == mp.MPCG_OK


def test_batched_outputs_must_not_overlap():
    import paper_2307_06072_amd as mp
    p0, p1 = _prob(0), list(_prob(1))
    p1[5] = p0[5]  # both problems write the same C
    assert _batch_call([p0, tuple(p1)]) == mp.MPCG_EINVAL
    assert "overlap" in mp.mpcg_last_error()
    p2 = list(_prob(2))
    p2[5] = p0[3]  # problem 2 writes problem 0's A
    assert _batch_call([p0, tuple(p2)]) == mp.MPCG_EINVAL


def test_max_spread_option_validated():
    import paper_2307_06072_amd as mp
    assert _call(opt=mp.mpcg_options(0, 0, 0, 0, -1)) == mp.MPCG_EINVAL
    assert _call(opt=mp.mpcg_options(0, 0, 0, 0, 1 << 25)) == mp.MPCG_EINVAL


def test_accumulate_validation():
    """mp_cgemm_acc validates like mp_cgemm_ex, plus its sign and slice type,
    before any device work."""
    import paper_2307_06072_amd as mp
    A, B, C = _fake_cmat(1 << 40), _fake_cmat(2 << 40), _fake_cmat(3 << 40)

    def acc(sign=-1, opt=None, m=4, ldc=4, Cm=C):
        return mp.mp_cgemm_acc_raw(m, 4, 4, ctypes.byref(A), 4, ctypes.byref(B), 4, ctypes.byref(Cm), ldc, 256, 1, 0,
                                   sign, ctypes.byref(opt) if opt is not None else None, None)

    for bad in (0, 2, -2):
        assert acc(sign=bad) == mp.MPCG_EINVAL
        assert "sign" in mp.mpcg_last_error()
    assert acc(ldc=3) == mp.MPCG_EINVAL
    assert acc(opt=mp.mpcg_options(mp.MPCG_SLICE_FP64, 0, 0, 0)) == mp.MPCG_EUNSUPPORTED
    Cbad = _fake_cmat(3 << 40)
    Cbad.re.sign = A.im.sign + 4  # the output overlaps an input
    assert acc(Cm=Cbad) == mp.MPCG_EINVAL
    assert acc(m=0) == 0


def test_batched_accumulate_validation():
    import paper_2307_06072_amd as mp
    arr = (mp.mpcg_problem * 1)()
    assert mp.mp_cgemm_batched_acc_raw(1, arr, 256, 1, 0, 0) == mp.MPCG_EINVAL
    assert "sign" in mp.mpcg_last_error()
    assert mp.mp_cgemm_batched_acc_raw(0, arr, 256, 1, 0, -1) == 0  # empty batch


# ---------------------------------------------------------------------------
# the multi-component input codec: host-side validation
# ---------------------------------------------------------------------------
def _codec(rows=4, cols=3, ncomp=2, src=7 << 40, ld=4, plane=0, dst=True, ldd=4, p=128, dst_part=None):
    import paper_2307_06072_amd as mp
    part = dst_part if dst_part is not None else mp.mpcg_part(8 << 40, (8 << 40) + (1 << 24), (8 << 40) + (2 << 24), 0)
    return mp._lib.mpcg_from_doubles(rows, cols, ncomp, src, ld, plane, ctypes.byref(part) if dst else None, ldd, p)


@pytest.mark.parametrize("kw", [dict(rows=-1), dict(cols=-2), dict(ncomp=0), dict(ncomp=5), dict(p=1),
                                dict(p=4097), dict(ld=3), dict(ldd=3), dict(src=0), dict(dst=False),
                                dict(plane=11)])
def test_codec_rejects_bad_arguments(kw):
    import paper_2307_06072_amd as mp
    assert _codec(**kw) == mp.MPCG_EINVAL
    assert mp.mpcg_last_error()


def test_codec_rejects_dst_overlapping_src():
    import paper_2307_06072_amd as mp
    src = 9 << 40
    # dst's exponent array inside the source doubles
    part = mp.mpcg_part(8 << 40, src + 16, (8 << 40) + (2 << 24), 0)
    assert _codec(src=src, dst_part=part) == mp.MPCG_EINVAL
    assert "overlap" in mp.mpcg_last_error()


# ---------------------------------------------------------------------------
# blocked LU entry points: argument errors found on the host
# ---------------------------------------------------------------------------
def _getrf(n=4, lda=4, ipiv=9 << 40, nb=2, p=256, mode=1, A=None):
    import paper_2307_06072_amd as mp
    A = _fake_cmat(1 << 40) if A is None else A
    return mp._lib.mp_zgetrf(n, ctypes.byref(A) if A is not False else None, lda, ipiv, nb, p, mode)


@pytest.mark.parametrize("kw", [dict(n=-1), dict(lda=3), dict(ipiv=0), dict(nb=-1), dict(p=1), dict(p=4097),
                                dict(mode=3), dict(A=False)])
def test_getrf_rejects_bad_arguments(kw):
    import paper_2307_06072_amd as mp
    assert _getrf(**kw) == mp.MPCG_EINVAL
    assert mp.mpcg_last_error()


def test_getrf_rejects_ipiv_inside_a():
    import paper_2307_06072_amd as mp
    assert _getrf(ipiv=(1 << 40) + (1 << 24) + 8) == mp.MPCG_EINVAL  # inside A.re's exponents
    assert "ipiv" in mp.mpcg_last_error()


def test_getrf_getrs_empty_is_a_no_op():
    import paper_2307_06072_amd as mp
    assert _getrf(n=0, lda=1) == 0
    A, B = _fake_cmat(1 << 40), _fake_cmat(2 << 40)
    assert mp._lib.mp_zgetrs(0, 3, ctypes.byref(A), 1, None, ctypes.byref(B), 1, 256, 1) == 0
    assert mp._lib.mp_zgetrs(4, 0, ctypes.byref(A), 4, 9 << 40, ctypes.byref(B), 4, 256, 1) == 0


@pytest.mark.parametrize("kw", [dict(n=-1), dict(nrhs=-1), dict(lda=3), dict(ldb=3), dict(ipiv=0), dict(B=False),
                                dict(p=1), dict(mode=5)])
def test_getrs_rejects_bad_arguments(kw):
    import paper_2307_06072_amd as mp
    args = dict(n=4, nrhs=2, lda=4, ipiv=9 << 40, ldb=4, p=256, mode=1, B=None)
    args.update(kw)
    A = _fake_cmat(1 << 40)
    B = _fake_cmat(2 << 40) if args["B"] is None else args["B"]
    st = mp._lib.mp_zgetrs(args["n"], args["nrhs"], ctypes.byref(A), args["lda"], args["ipiv"],
                           ctypes.byref(B) if B is not False else None, args["ldb"], args["p"], args["mode"])
    assert st == mp.MPCG_EINVAL


def test_getrs_rejects_b_overlapping_a():
    import paper_2307_06072_amd as mp
    A = _fake_cmat(1 << 40)
    assert mp._lib.mp_zgetrs(4, 2, ctypes.byref(A), 4, 9 << 40, ctypes.byref(A), 4, 256, 1) == mp.MPCG_EINVAL
    assert "overlap" in mp.mpcg_last_error()


def test_adaptive_option_validated():
    import paper_2307_06072_amd as mp
    for bad in (2, -1, 48, 1 << 21):
        assert _call(opt=mp.mpcg_options(0, 0, 0, 0, 0, bad)) == mp.MPCG_EINVAL
        assert "adaptive" in mp.mpcg_last_error()


# ---------------------------------------------------------------------------
# size-class tuning cache (file side; no GPU needed)
# ---------------------------------------------------------------------------
def test_tune_cache_file_round_trip(tmp_path, monkeypatch):
    """A cache file is read back entry for entry after a save; a malformed or
    missing file and a missing path are rejected with MPCG_EINVAL.  Without a
    GPU the device's architecture reads as "unknown", so the file is written
    for that name here."""
    import json
    import torch
    import paper_2307_06072_amd as mp
    if torch.cuda.is_available():
        pytest.skip("the file names this host's architecture only when there is no GPU (the GPU tuning test covers it)")
    monkeypatch.delenv("MPCG_TUNE_CACHE", raising=False)
    mp.mpcg_tune_clear()
    entries = [{"arch": "unknown", "scheme": 0, "mode": 2, "log2_m": 9, "log2_n": 8, "log2_k": 10, "s_bucket": 5,
                "band": 12, "groups": 1024, "mode3m": 0, "us": 123.5},
               {"arch": "unknown", "scheme": 1, "mode": 1, "log2_m": 11, "log2_n": 11, "log2_k": 11,
                "s_bucket": 20, "band": 20, "groups": 512, "mode3m": 1, "us": 240000.0},
               {"arch": "gfx000", "scheme": 0, "mode": 1, "log2_m": 4, "log2_n": 4, "log2_k": 4, "s_bucket": 5,
                "band": 8, "groups": 256, "mode3m": 1, "us": 5.0}]
    src = tmp_path / "cache.json"
    src.write_text(json.dumps({"mpcg_tune_cache": 1, "entries": entries}))
    assert mp.mpcg_tune_load(str(src)) == 2  # the other architecture's entry is skipped
    out = tmp_path / "out.json"
    assert mp.mpcg_tune_save(str(out)) == 2
    got = json.loads(out.read_text())
    assert got["mpcg_tune_cache"] == 1
    key = lambda e: (e["scheme"], e["mode"], e["log2_m"], e["log2_n"], e["log2_k"], e["s_bucket"])
    assert sorted(got["entries"], key=key) == sorted(entries[:2], key=key)
    bad = tmp_path / "bad.json"
    bad.write_text('{"mpcg_tune_cache": 1, "entries": [{"arch": "unknown", "band": 7}]}')
    for path in (str(bad), str(tmp_path / "missing.json")):
        with pytest.raises(mp.MPCGError) as ei:
            mp.mpcg_tune_load(path)
        assert ei.value.code == mp.MPCG_EINVAL
    with pytest.raises(mp.MPCGError) as ei:
        mp.mpcg_tune_load(None)
    assert ei.value.code == mp.MPCG_EINVAL
    monkeypatch.setenv("MPCG_TUNE_CACHE", str(out))
    mp.mpcg_tune_clear()
    assert mp.mpcg_tune_load(None) == 2
    mp.mpcg_tune_clear()


def test_auto_mode_accepted_bad_mode_rejected():
    import paper_2307_06072_amd as mp
    assert _call(mode=3) == mp.MPCG_EINVAL
    assert _call(mode=mp.MPCG_AUTO) != mp.MPCG_EINVAL  # passes validation; fails later without a GPU


@pytest.mark.parametrize("kind,blocks,iters,null", [(2, 8, 8, None), (-1, 8, 8, None), (0, 0, 8, None),
                                                   (0, (1 << 20) + 1, 8, None), (1, 8, 0, None),
                                                   (1, 8, (1 << 24) + 1, None), (0, 8, 8, "sink"),
                                                   (0, 8, 8, "ops"), (1, 8, 8, "ms")])
def test_probe_rejects_bad_arguments(kind, blocks, iters, null):
    """The matrix-core probe checks its arguments before any device work."""
    import paper_2307_06072_amd as mp
    lib = ctypes.CDLL(mp.LIB_PATH)
    lib.mpcg_probe_mfma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)]
    ops, ms = ctypes.c_double(0.0), ctypes.c_float(0.0)
    sink = None if null == "sink" else ctypes.c_void_p(1 << 40)
    rc = lib.mpcg_probe_mfma(kind, blocks, iters, sink, None if null == "ops" else ctypes.byref(ops),
                             None if null == "ms" else ctypes.byref(ms))
    assert rc == mp.MPCG_EINVAL
