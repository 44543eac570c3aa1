"""Size-class tuning: mpcg_autotune measures plans, stores the fastest, and
the planner then uses it; results stay bit-identical to the oracle (exact
scheme), for single products, the automatic form and batches; the cache
survives a save, clear and load."""
from __future__ import annotations

import json
import sys

import pytest

import oracle
from mpgen import random_cmat
from tests.gpu_util import device_result_to_host, mismatches

pytestmark = pytest.mark.gpu

M4, M3, AUTO = 0, 1, 2
EXACT = 0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_autotune_then_tuned_calls_are_exact(tmp_path):
    import torch
    import paper_2307_06072_amd as mp
    mp.mpcg_tune_clear()
    m, n, k, p = 96, 80, 130, 256
    A = random_cmat(97, 0, m, k, p, 6)
    B = random_cmat(97, 1, k, n, p, 6)
    ref = oracle.cgemm(A, B, p)
    dA, dB = mp.to_device(A), mp.to_device(B)
    C = mp.device_empty(m, n, p)
    mp.mpcg_set_stream()
    _say("autotune 96 x 80 x 130, 256 bits, AUTO")
    rep = mp.mpcg_autotune(m, n, k, dA, m, dB, k, C, m, p, AUTO, EXACT, reps=1)
    _say(f"choice {rep}")
    assert rep["band"] in (8, 12, 16, 20) and rep["groups"] in (256, 512, 1024, 2048)
    assert rep["mode"] in (M4, M3) and rep["candidates"] >= 16
    assert 0 < rep["us"] <= rep["untuned_us"]
    # the tuned plan is the one used, and it is exact
    for mode in (AUTO, rep["mode"]):
        C2 = mp.device_empty(m, n, p)
        info = mp.mp_cgemm_ex(m, n, k, dA, m, dB, k, C2, m, p, mode, EXACT)
        torch.cuda.synchronize()
        assert mp.mpcg_stream_status() == 0
        if mode == AUTO:
            assert info["block"] == rep["band"] and info["nprod"] == (3 if rep["mode"] == M3 else 4)
        bad, first = mismatches(device_result_to_host(C2, p), ref, m, n)
        assert bad == 0, (mode, first)
    path = tmp_path / "tune.json"
    assert mp.mpcg_tune_save(str(path)) == 1
    entries = json.loads(path.read_text())["entries"]
    assert entries[0]["band"] == rep["band"] and entries[0]["mode3m"] == (1 if rep["mode"] == M3 else 0)
    mp.mpcg_tune_clear()
    assert mp.mpcg_tune_load(str(path)) == 1
    mp.mpcg_tune_clear()


def test_tuned_batch_is_exact():
    """A batch whose problems fall in tuned size classes (with the automatic
    form) runs each class's band and form in its own launch; every product is
    still the oracle's."""
    import torch
    import paper_2307_06072_amd as mp
    mp.mpcg_tune_clear()
    p = 200
    shapes = [(40, 50, 70), (120, 90, 64), (40, 52, 66), (200, 16, 130)]
    batch = []
    for t, (m, n, k) in enumerate(shapes):
        A = random_cmat([98, t], 0, m, k, p, 5)
        B = random_cmat([98, t], 1, k, n, p, 5)
        batch.append((m, n, k, A, B))
    mp.mpcg_set_stream()
    for (m, n, k, A, B) in batch[:2]:  # tune two classes
        dA, dB, C = mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)
        _say(f"autotune {m} x {n} x {k}")
        mp.mpcg_autotune(m, n, k, dA, m, dB, k, C, m, p, AUTO, EXACT, reps=1)
    devs = [(mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)) for (m, n, k, A, B) in batch]
    _say("tuned batch")
    mp.mp_cgemm_batched(devs, p, AUTO, EXACT)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    for (m, n, k, A, B), (_, _, C) in zip(batch, devs):
        bad, first = mismatches(device_result_to_host(C, p), oracle.cgemm(A, B, p), m, n)
        assert bad == 0, (m, n, k, first)
    mp.mpcg_tune_clear()


def test_autotune_batched_choice_is_used_and_exact():
    import torch
    import paper_2307_06072_amd as mp
    mp.mpcg_tune_clear()
    p = 256
    shapes = [(64, 64, 64), (100, 40, 200), (33, 90, 120), (128, 16, 300), (70, 70, 70), (20, 200, 50)]
    batch = []
    for t, (m, n, k) in enumerate(shapes):
        batch.append((m, n, k, random_cmat([99, t], 0, m, k, p, 8), random_cmat([99, t], 1, k, n, p, 8)))
    devs = [(mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)) for (m, n, k, A, B) in batch]
    mp.mpcg_set_stream()
    _say("autotune batched")
    rep = mp.mpcg_autotune_batched(devs, p, AUTO, EXACT, reps=1)
    _say(f"batch choice {rep}")
    assert rep["candidates"] == 7 and rep["untuned_us"] > 0 and rep["us"] <= rep["untuned_us"]
    assert rep["band"] in (0, 8, 12, 16, 20)
    for (_, _, C) in devs:
        for part in (C.re, C.im):
            part.exp.fill_(3)
    info = mp.mp_cgemm_batched(devs, p, AUTO, EXACT)
    torch.cuda.synchronize()
    assert mp.mpcg_stream_status() == 0
    if rep["band"]:
        assert info["block"] == rep["band"]
        assert info["nprod"] == (3 if rep["mode"] == M3 else 4)
    for (m, n, k, A, B), (_, _, C) in zip(batch, devs):
        bad, first = mismatches(device_result_to_host(C, p), oracle.cgemm(A, B, p), m, n)
        assert bad == 0, (m, n, k, first)
    mp.mpcg_tune_clear()
