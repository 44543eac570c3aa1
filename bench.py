#!/usr/bin/env python3
"""Benchmark of the Ozaki-scheme multi-precision complex GEMM on one MI355X.

Default workload: C = AB with m = n = k = 2048 at 1024-bit precision,
exponents uniform on [-32, 32] (INT8 slices, 3M form, exact scheme).  A step
is one whole mp_cgemm call (exponent scan, split, slice GEMM, rounding) with
the inputs already resident in HBM.  Prints ONE JSON line on stdout; progress
goes to stderr.

Also reported in "extra": the 512^3 / 512-bit family (FP64-slice 4M vs
INT8-slice 4M vs INT8-slice 3M, exact and truncated) with the INT8-3M over
FP64-4M speedup, the truncated scheme on the default workload, a batch of
256 products, the LU trailing-update stream, the blocked LU of order 4096
(block 128, 256 bits, A + n(1+i)I, b = A(1+i) ones) and the
multi-component codec.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MP complex GEMM 8mnk/s at 256/1024-bit; INT8-3M vs FP64-4M Ozaki speedup"
PEAK_INT8_TOPS = 5000.0   # MI355X dense INT8 matrix peak, TOP/s
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 matrix peak, TFLOP/s
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E, GB/s
M3_MODE = 1


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _mode(s):
    import paper_2307_06072_amd as mp
    return {"3M": mp.MPCG_3M, "4M": mp.MPCG_4M}[s]


def _scheme(s):
    import paper_2307_06072_amd as mp
    return {"exact": mp.MPCG_EXACT, "truncated": mp.MPCG_TRUNCATED}[s]


def _slice(s):
    import paper_2307_06072_amd as mp
    return {"int8": mp.MPCG_SLICE_INT8, "fp64": mp.MPCG_SLICE_FP64}[s]


def time_calls(dA, dB, dC, m, n, k, p, mode, scheme, slice_type, steps, warmup, strassen=0):
    """Warm up, then time `steps` whole calls; returns (seconds, info, avg stage us)."""
    import torch
    import paper_2307_06072_amd as mp
    mp.mpcg_set_stream()
    info = None
    for _ in range(warmup):
        info = mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mode, scheme, slice_type=slice_type,
                              strassen=strassen)
    torch.cuda.synchronize()
    mp.mpcg_enable_timing(True)
    mp.mpcg_timing_report()  # start a fresh collection
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mode, scheme, slice_type=slice_type,
                              strassen=strassen)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    us_sum, ncalls = mp.mpcg_timing_report()
    mp.mpcg_enable_timing(False)
    st = mp.mpcg_stream_status()
    if st != 0:
        raise RuntimeError(f"device status {st}: {mp.mpcg_last_error()}")
    avg = [u / max(1, ncalls) for u in us_sum]
    return t1 - t0, info, avg


def stage_bytes(m, n, k, p, info, mode3m, slice_fp64):
    """Algorithmic HBM bytes of the split and round stages (per call).  With
    one level of Strassen's recursion the split reads 12 operand quadrants per
    side (three whole operands) and writes 7 quarter-size slice sets, and the
    rounding reads 12 quarter-size product streams (three whole ones) per
    contraction chunk."""
    L = (p + 63) // 64
    esz = 8 if slice_fp64 else 1
    ent_in = 2 * (8 * L + 5)  # Re + Im: limbs, exponent, sign
    nops_a = 3 if mode3m else 2
    nops_b = 3
    rd, wr = (3.0, 7.0 / 4.0) if info.get("strassen") else (1.0, 1.0)
    split = (m * k + k * n) * ent_in * rd + (m * k * nops_a * info["S_A"] + k * n * nops_b * info["S_B"]) * esz * wr
    nd = info["cutoff"] + 1
    dig = 4 if slice_fp64 else 1
    rnd = m * n * 2 * (nd * dig * info["ksplit"] + 12) * rd + m * n * ent_in
    return split, rnd


def mfma_probe(kind: int, target_ms: float = 300.0):
    """Register-only rate of a slice product's matrix instruction (kind 0:
    INT8 v_mfma_i32_16x16x64_i8, 1: FP64 v_mfma_f64_16x16x4_f64), 8
    workgroups of 4 wavefronts per compute unit: the best of three runs of
    about target_ms (long enough for the clock to settle under the load, as
    it does under the slice GEMM), in TOP/s (TFLOP/s for FP64), and the
    run's shape."""
    import torch
    import paper_2307_06072_amd as mp
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    blocks, iters = 256 * 8, 256
    mp.mpcg_set_stream()
    mp.mpcg_probe_mfma(kind, blocks, iters, sink.data_ptr())  # warm-up
    _, ms = mp.mpcg_probe_mfma(kind, blocks, iters, sink.data_ptr())
    iters = max(1, min(1 << 24, int(iters * target_ms / max(ms, 1e-3))))
    best = 0.0
    for _ in range(3):
        ops, ms = mp.mpcg_probe_mfma(kind, blocks, iters, sink.data_ptr())
        best = max(best, ops / (ms * 1e-3) / 1e12)
    return best, {"blocks": blocks, "workgroup_threads": 256, "iters": iters, "instructions_per_iter": 8}


def traffic_record(kernel_src: str, form: str):
    """HBM traffic per launch of the slice GEMM from committed rocprofv3
    counters, if they were taken on the current kernel source in this form
    ("plain" or "strassen1", whose launches are half-size products), else None."""
    path = os.path.join(ROOT, "profiles", f"gemm_i8_traffic_{form}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(kernel_src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if rec.get("source_sha256") != sha or rec.get("form") != form:
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_baseline(A, B, m, n, k, p, target_s):
    """The oracle on a bounded sample of output entries, all host threads."""
    import numpy as np
    import oracle
    threads = oracle.default_threads()
    rng = np.random.default_rng(12345)
    # calibrate on growing samples until one takes at least a second
    probe = max(threads, 8)
    while True:
        rows = rng.integers(0, m, probe)
        cols = rng.integers(0, n, probe)
        t0 = time.perf_counter()
        oracle.cgemm_entries(A, B, rows, cols, p, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= 1.0 or probe >= m * n:
            break
        probe = min(m * n, probe * 4)
    per = dt / probe
    nent = int(max(threads, min(m * n, target_s / max(per, 1e-9))))
    rows = rng.integers(0, m, nent)
    cols = rng.integers(0, n, nent)
    log(f"cpu baseline: oracle on {nent} entries with {threads} threads")
    t0 = time.perf_counter()
    oracle.cgemm_entries(A, B, rows, cols, p, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": 8.0 * k * nent / dt, "unit": "8mnk/s", "cores": threads, "kind": "oracle",
            "sample": f"{nent} random output entries (both components) of the {m}x{n}x{k} product, "
                      f"{dt:.1f} s wall on {threads} threads; value = 8*k*entries/s"}


def small_latency_case():
    """64^3 at 256 bits: FP64-4M (the paper's plain form) and INT8-3M, exact."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import workload_inputs
    log("64^3 at 256 bits")
    m, n, k, p, A, B = workload_inputs("cgemm64_p256")
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)
    out = {}
    for sl, md in (("fp64", "4M"), ("int8", "3M")):
        dt, info, st = time_calls(dA, dB, dC, m, n, k, p, _mode(md), _scheme("exact"), _slice(sl), steps=20, warmup=3)
        out[f"{sl}_{md}_exact"] = {"ms_per_call": 1000 * dt / 20, "8mnk_per_s": 8.0 * m * n * k * 20 / dt,
                                   "stage_us": st, "S_A": info["S_A"], "pairs": info["pairs"]}
    # one-call latency of tiny products (timing events off)
    lat = {}
    for (mm, nn, kk) in ((1, 1, 1), (16, 16, 16), (64, 64, 64)):
        from mpgen import random_cmat
        A1 = random_cmat(3, 0, mm, kk, p, 4)
        B1 = random_cmat(3, 1, kk, nn, p, 4)
        d1, d2, d3 = mp.to_device(A1), mp.to_device(B1), mp.device_empty(mm, nn, p)
        mp.mpcg_set_stream()
        for _ in range(10):
            mp.mp_cgemm_ex(mm, nn, kk, d1, d1.ld, d2, d2.ld, d3, d3.ld, p, mp.MPCG_3M, mp.MPCG_EXACT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            mp.mp_cgemm_ex(mm, nn, kk, d1, d1.ld, d2, d2.ld, d3, d3.ld, p, mp.MPCG_3M, mp.MPCG_EXACT)
        torch.cuda.synchronize()
        lat[f"{mm}x{nn}x{kk}"] = 1e6 * (time.perf_counter() - t0) / 50
    out["int8_3M_exact_latency_us"] = lat
    return {"cgemm64_p256": out}


def f64_case(calls=3):
    """The FP64 plain form on the 512^3 / 512-bit workload (4M exact), `calls`
    calls (for profiling the DGEMMs and the accumulation)."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import workload_inputs
    m, n, k, p, A, B = workload_inputs("cgemm512_p512")
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)
    mp.mpcg_set_stream()
    t0 = time.perf_counter()
    for _ in range(calls):
        info = mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mp.MPCG_4M, mp.MPCG_EXACT,
                              slice_type=mp.MPCG_SLICE_FP64)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / calls
    if mp.mpcg_stream_status() != 0:
        raise RuntimeError(mp.mpcg_last_error())
    return {"fp64_4M_exact_512": {"calls": calls, "ms_per_call_incl_first": 1000 * dt, "S_A": info["S_A"],
                                  "pairs": info["pairs"]}}


def batched_case():
    """256 independent products, shapes uniform on [16, 768]^3, 256 bits,
    exponents in [-8, 8]: one mp_cgemm_batched call against one call each."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import batched_inputs
    log("batched: 256 uneven products at 256 bits")
    p = 256
    batch = batched_inputs(256, 4, p, 8)
    devs = [(mp.to_device(A), mp.to_device(B), mp.device_empty(m, n, p)) for (m, n, k, A, B) in batch]
    del batch
    work = sum(8.0 * A.rows * B.cols * A.cols for (A, B, _) in devs)
    mp.mpcg_set_stream()
    info = mp.mp_cgemm_batched(devs, p, mp.MPCG_3M)
    torch.cuda.synchronize()
    mp.mpcg_enable_timing(True)
    mp.mpcg_timing_report()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        info = mp.mp_cgemm_batched(devs, p, mp.MPCG_3M)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    us, nc = mp.mpcg_timing_report()
    mp.mpcg_enable_timing(False)
    st = [u / max(1, nc) for u in us]
    t0 = time.perf_counter()
    for (dA, dB, dC) in devs:
        mp.mp_cgemm(dA.rows, dB.cols, dA.cols, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mp.MPCG_3M, mp.MPCG_EXACT)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    if mp.mpcg_stream_status() != 0:
        raise RuntimeError(mp.mpcg_last_error())
    # the same batch planned from a spread bound (exponents on [-8, 8]: spread
    # at most 16), captured once into a HIP graph and replayed
    bound = 16
    wsz = mp.mpcg_workspace_size_batched(devs, p, mp.MPCG_3M, mp.MPCG_EXACT, max_spread=bound)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    mp.mpcg_set_workspace(ws.data_ptr(), wsz)
    try:
        mp.mp_cgemm_batched(devs, p, mp.MPCG_3M, mp.MPCG_EXACT, max_spread=bound)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                mp.mpcg_set_stream(side.cuda_stream)
                infog = mp.mp_cgemm_batched(devs, p, mp.MPCG_3M, mp.MPCG_EXACT, max_spread=bound)
        mp.mpcg_set_stream()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t0) / reps
        if mp.mpcg_stream_status() != 0:
            raise RuntimeError(mp.mpcg_last_error())
    finally:
        mp.mpcg_set_workspace(None, 0)
        mp.mpcg_set_stream()
    del ws
    log(f"  one call {1000 * dt:.1f} ms, graph replay {1000 * dtg:.1f} ms")
    # size-class tuning: one representative (the most work) per class of
    # (ceil log2 m, n, k), every plan measured once, the form left to the tuner;
    # then the batch with the tuned plans, its bits checked against the untuned run
    import math
    tuned = tune_batch(devs, p)
    before = [(C.re.mant.clone(), C.im.mant.clone(), C.re.exp.clone(), C.im.exp.clone()) for (_, _, C) in devs]
    infot = mp.mp_cgemm_batched(devs, p, mp.MPCG_AUTO)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        infot = mp.mp_cgemm_batched(devs, p, mp.MPCG_AUTO)
    torch.cuda.synchronize()
    dtt = (time.perf_counter() - t0) / reps
    same = all(torch.equal(a, C.re.mant) and torch.equal(b, C.im.mant) and torch.equal(c, C.re.exp) and
               torch.equal(d, C.im.exp) for (a, b, c, d), (_, _, C) in zip(before, devs))
    mp.mpcg_tune_clear()
    if mp.mpcg_stream_status() != 0 or not same:
        raise RuntimeError(f"tuned batch: status {mp.mpcg_last_error()}, identical bits {same}")
    log(f"  tuned ({tuned['batch_choice']}, {tuned['seconds']:.1f} s): batch {1000 * dtt:.1f} ms")
    return {"batched256_p256": {"ms_per_call": 1000 * dt, "8mnk_per_s": work / dt, "stage_us": st,
                                "gemm_frac_of_peak": info["algo_ops"] / (st[2] * 1e-6) / 1e12 / PEAK_INT8_TOPS,
                                "one_call_each_ms": 1000 * dt1, "speedup_over_one_call_each": dt1 / dt,
                                "pairs_total": info["pairs"], "block": info["block"],
                                "graph_ms_per_replay": 1000 * dtg, "graph_8mnk_per_s": work / dtg,
                                "graph_max_spread": bound, "graph_pairs_total": infog["pairs"],
                                "graph_workspace_bytes": wsz,
                                "tuned_ms_per_call": 1000 * dtt, "tuned_8mnk_per_s": work / dtt,
                                "tuned_identical_bits": same, "tuned_pairs_total": infot["pairs"],
                                "tuner": tuned}}


def tune_batch(devs, p):
    """mpcg_autotune_batched on the whole batch (every band width and both
    forms measured on the batch itself, one timed call each), then
    mpcg_autotune on one representative per size class of (ceil log2 m, n,
    k), the class's largest product, for the single-call choices.  The batch
    is then timed with MPCG_AUTO, which takes the batch tuner's choice.
    Returns the choices and the tuning time."""
    import math
    import paper_2307_06072_amd as mp
    mp.mpcg_tune_clear()
    t0 = time.perf_counter()
    classes = {}
    for (A, B, C) in devs:
        key = tuple(max(0, math.ceil(math.log2(max(1, v)))) for v in (A.rows, B.cols, A.cols))
        if key not in classes or A.rows * B.cols * A.cols > classes[key][0]:
            classes[key] = (A.rows * B.cols * A.cols, (A, B, C))
    single = {}
    for key, (_, (A, B, C)) in sorted(classes.items()):
        r = mp.mpcg_autotune(A.rows, B.cols, A.cols, A, A.ld, B, B.ld, C, C.ld, p, mp.MPCG_AUTO, mp.MPCG_EXACT, reps=1)
        k = f"{'3M' if r['mode'] == mp.MPCG_3M else '4M'} band {r['band']}"
        single[k] = single.get(k, 0) + 1
    t1 = time.perf_counter()
    # the batch tuner runs last: its choice replaces the single-call entries of the classes it covers
    rb = mp.mpcg_autotune_batched(devs, p, mp.MPCG_AUTO, mp.MPCG_EXACT, reps=1)
    return {"seconds": time.perf_counter() - t0, "single_call_classes": len(classes),
            "single_call_seconds": t1 - t0, "single_call_choices": single,
            "batch_choice": ("per-problem rule kept" if rb["band"] == 0 else
                             f"{'3M' if rb['mode'] == mp.MPCG_3M else '4M'} band {rb['band']}"),
            "batch_candidates": rb["candidates"], "batch_tuned_ms": rb["us"] / 1000,
            "batch_untuned_ms": rb["untuned_us"] / 1000}


def codec_case():
    """Multi-component inputs: a 2048 x 2048 complex matrix given as
    quad-double components (four doubles per real component, a normalised
    expansion), converted to 256 bits by mpcg_from_doubles and back by
    mpcg_to_doubles (HBM-bound: 64 B of doubles and 74 B of the number format
    per complex entry)."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import multi_double
    log("codec: 2048 x 2048 quad-double -> 256 bits")
    rows = cols = 2048
    p, nc = 256, 4
    re = torch.from_numpy(multi_double(7, 0, nc, rows, cols, "expansion", 60)).cuda()
    im = torch.from_numpy(multi_double(7, 1, nc, rows, cols, "expansion", 60)).cuda()
    mp.mpcg_set_stream()
    C = mp.from_doubles(re, im, p)
    torch.cuda.synchronize()

    def issue():
        for t, part in ((re, C.re), (im, C.im)):
            mp._check(mp.mpcg_from_doubles(rows, cols, nc, t.data_ptr(), rows, rows * cols, part, C.ld, p))
    issue()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        issue()
    e1.record()
    torch.cuda.synchronize()
    if mp.mpcg_stream_status() != 0:
        raise RuntimeError(mp.mpcg_last_error())
    ms = e0.elapsed_time(e1) / reps
    # and back: the same matrix as quad-double components
    outs = [torch.empty_like(re), torch.empty_like(im)]

    def issue_back():
        for t, part in zip(outs, (C.re, C.im)):
            mp._check(mp.mpcg_to_doubles(rows, cols, part, C.ld, p, nc, t.data_ptr(), rows, rows * cols))
    issue_back()
    e0.record()
    for _ in range(reps):
        issue_back()
    e1.record()
    torch.cuda.synchronize()
    if mp.mpcg_stream_status() != 0:
        raise RuntimeError(mp.mpcg_last_error())
    ms_back = e0.elapsed_time(e1) / reps
    L = (p + 63) // 64
    nbytes = rows * cols * 2 * (nc * 8 + 1 + 4 + 8 * L)
    return {"codec_qd2048_p256": {"ms_per_call": ms, "entries_per_s": rows * cols / (ms * 1e-3),
                                  "algorithmic_GBps": nbytes / (ms * 1e-3) / 1e9,
                                  "to_doubles_ms_per_call": ms_back,
                                  "to_doubles_algorithmic_GBps": nbytes / (ms_back * 1e-3) / 1e9,
                                  "hbm_peak_GBps": PEAK_HBM_GBS}}


def adaptive_case(A, B, p):
    """Adaptive slicing on the 2048 workload with mixed spreads: rows 1536..2047
    of A and columns 1536..2047 of B each get one entry raised by 2^300, so a
    quarter of the rows and columns need S = 199 slices while the rest need
    156.  One plan for the whole product against slice counts per block
    (mpcg_options.adaptive); the bits are compared on the device."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import EXP_ZERO
    log("adaptive slicing: 2048^3, 1024 bits, a quarter of the rows/columns 300 bits wider")
    A, B = A.copy(), B.copy()
    m, k, n = A.rows, A.cols, B.cols
    for r in range(3 * m // 4, m):
        if A.re.exp[3, r] != EXP_ZERO:
            A.re.exp[3, r] += 300
    for c in range(3 * n // 4, n):
        if B.re.exp[c, 5] != EXP_ZERO:
            B.re.exp[c, 5] += 300
    dA, dB = mp.to_device(A), mp.to_device(B)
    out, res = {}, []
    mp.mpcg_set_stream()
    for adaptive in (0, 1):
        dC = mp.device_empty(m, n, p)
        info = mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mp.MPCG_3M, mp.MPCG_EXACT, adaptive=adaptive)
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mp.MPCG_3M, mp.MPCG_EXACT, adaptive=adaptive)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        if mp.mpcg_stream_status() != 0:
            raise RuntimeError(mp.mpcg_last_error())
        out["adaptive" if adaptive else "one_plan"] = {"ms_per_call": 1000 * dt, "8mnk_per_s": 8.0 * m * n * k / dt,
                                                      "max_S_A": info["S_A"], "algo_ops": info["algo_ops"]}
        res.append(dC)
        log(f"  adaptive={adaptive}: {1000 * dt:.1f} ms")
    same = all(torch.equal(getattr(getattr(res[0], h), f), getattr(getattr(res[1], h), f))
               for h in ("re", "im") for f in ("sign", "exp", "mant"))
    out["identical_bits"] = bool(same)
    out["speedup"] = out["one_plan"]["ms_per_call"] / out["adaptive"]["ms_per_call"]
    return {"cgemm2048_p1024_mixed_spread": out}


def parts_case():
    """Separate Re/Im scales on the 2048 workload at 1024 bits with every
    imaginary part 2^200 below the real parts: one scale per row in 4M and 3M
    (the slices cover the 200-bit gap) against the part_scales option in 4M;
    the bits are compared on the device."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import workload_inputs
    log("separate Re/Im scales: 2048^3, 1024 bits, Im parts 2^-200 below Re")
    m, n, k, p, A, B = workload_inputs("cgemm2048_p1024_im200")
    dA, dB = mp.to_device(A), mp.to_device(B)
    del A, B
    out, res = {}, []
    mp.mpcg_set_stream()
    for key, mode, parts in (("one_scale_4M", mp.MPCG_4M, 0), ("one_scale_3M", mp.MPCG_3M, 0),
                             ("part_scales_4M", mp.MPCG_4M, 1)):
        dC = mp.device_empty(m, n, p)
        info = mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mode, mp.MPCG_EXACT, part_scales=parts)
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            mp.mp_cgemm_ex(m, n, k, dA, dA.ld, dB, dB.ld, dC, dC.ld, p, mode, mp.MPCG_EXACT, part_scales=parts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        if mp.mpcg_stream_status() != 0:
            raise RuntimeError(mp.mpcg_last_error())
        out[key] = {"ms_per_call": 1000 * dt, "8mnk_per_s": 8.0 * m * n * k / dt, "S_A": info["S_A"],
                    "S_B": info["S_B"], "pairs": info["pairs"], "part_scales": info["part_scales"],
                    "gemm_frac_of_peak_est": info["algo_ops"] / dt / 1e12 / PEAK_INT8_TOPS}
        res.append(dC)
        log(f"  {key}: {1000 * dt:.1f} ms (S = {info['S_A']})")
    same = all(torch.equal(getattr(getattr(res[0], h), f), getattr(getattr(res[i], h), f))
               for i in (1, 2) for h in ("re", "im") for f in ("sign", "exp", "mant"))
    out["identical_bits"] = bool(same)
    out["speedup_over_one_scale_4M"] = out["one_scale_4M"]["ms_per_call"] / out["part_scales_4M"]["ms_per_call"]
    out["speedup_over_one_scale_3M"] = out["one_scale_3M"]["ms_per_call"] / out["part_scales_4M"]["ms_per_call"]
    return {"cgemm2048_p1024_im200": out}


def lu_full_case(n=4096, nb=128, p=256):
    """The blocked LU workload: A with random entries (exponents on [-2, 2])
    plus n (1 + i) on the diagonal (each shifted component rounded once, by
    one accumulating product on the diagonal viewed as a row with leading
    dimension lda + 1), b = A (1 + i) ones rounded
    once by mp_cgemm; mp_zgetrf with block width nb, then mp_zgetrs.  Reports
    the seconds of each and the largest relative error of x against
    (1 + i) ones (|Re| + |Im| norm)."""
    from fractions import Fraction
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import EXP_ZERO, random_cmat
    log(f"blocked LU n={n} nb={nb} p={p}: A + n(1+i)I, b = A (1+i) ones")
    L = (p + 63) // 64
    A = random_cmat([5, n], 0, n, n, p, 2)
    dA = mp.to_device(A)
    del A

    def scalar(vre, vim):  # a 1 x 1 matrix holding vre + i vim, both powers of two or zero
        M = mp.device_empty(1, 1, p)
        for part, v in ((M.re, vre), (M.im, vim)):
            if v:
                e = v.bit_length()
                assert v == 1 << (e - 1)
                part.exp.fill_(e)
                part.mant[L - 1].fill_(-(1 << 63))  # top bit only (uint64 pattern as int64)
        return M

    # the diagonal as a 1 x n row (leading dimension lda + 1) := itself + n(1+i) x (1 x n row of ones)
    dn = scalar(n, n)
    row1 = mp.device_empty(1, n, p)
    for part in (row1.re,):
        part.exp.fill_(1)
        part.mant[L - 1].fill_(-(1 << 63))
    diag = mp.DeviceCMat(1, n, dA.ld + 1, dA.L, dA.re, dA.im)
    mp.mpcg_set_stream()
    mp.mp_cgemm_acc(1, n, 1, dn, 1, row1, 1, diag, dA.ld + 1, p, +1)
    ones = mp.device_empty(n, 1, p)
    for part in (ones.re, ones.im):
        part.exp.fill_(1)
        part.mant[L - 1].fill_(-(1 << 63))
    dB = mp.device_empty(n, 1, p)
    mp.mp_cgemm(n, 1, n, dA, dA.ld, ones, ones.ld, dB, dB.ld, p)
    # warm-up of every kernel on a small case
    dW = mp.to_device(random_cmat([5, 16], 0, 16, 16, p, 2))
    wp = torch.zeros(16, dtype=torch.int32, device="cuda")
    mp.mp_zgetrf(16, dW, dW.ld, wp, 8, p, mp.MPCG_3M)
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = mp.mp_zgetrf(n, dA, dA.ld, ipiv, nb, p, mp.MPCG_3M)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"  getrf {t1 - t0:.2f} s")
    mp.mp_zgetrs(n, 1, dA, dA.ld, ipiv, dB, dB.ld, p, mp.MPCG_3M)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if info != 0 or mp.mpcg_stream_status() != 0:
        raise RuntimeError(f"LU failed: info {info}, {mp.mpcg_last_error()}")
    h = mp.to_numpy(dB)
    err = Fraction(0)
    for k in range(n):
        comps = []
        for name in ("re", "im"):
            sg, ex, mt = h[name]
            if ex[0, k] == EXP_ZERO:
                comps.append(Fraction(0))
                continue
            M = 0
            for l in range(L - 1, -1, -1):
                M = (M << 64) | int(mt[l, 0, k])
            v = Fraction(M) * Fraction(2) ** (int(ex[0, k]) - 64 * L)
            comps.append(-v if sg[0, k] else v)
        err = max(err, (abs(comps[0] - 1) + abs(comps[1] - 1)) / 2)
    log(f"  getrs {t2 - t1:.2f} s, max relative error {float(err):.2e}")
    pivots_moved = int((ipiv.cpu() != torch.arange(n, dtype=torch.int32)).sum())
    return {f"lu_full_n{n}_b{nb}_p{p}": {"getrf_s": t1 - t0, "getrs_s": t2 - t1, "max_rel_err": float(err),
                                         "rows_exchanged": pivots_moved,
                                         "matrix": "random (e in [-2, 2]) + n(1+i) I",
                                         "rhs": "b = A (1+i) ones"}}


def lu_paper_case(widths=(128,), precs=(256,)):
    """The paper's LU experiment (Sec. IV-B) at n = 1024 and 256 (512, 768)
    bits: A with random entries (exponents on [-2, 2]), x_k = k + k i, b = A x
    rounded once by mp_cgemm; mp_zgetrf with block width K, then mp_zgetrs.
    Reports the seconds of each and the largest relative error of x (|Re| +
    |Im| norm)."""
    rec = {}
    for p in precs:
        rec[f"lu_paper_n1024_p{p}"] = _lu_full_one(widths, p)
    return rec


def _lu_full_one(widths, p):
    from fractions import Fraction
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import EXP_ZERO, random_cmat
    n = 1024
    A = random_cmat([6, n], 0, n, n, p, 2)
    L = (p + 63) // 64
    xs = random_cmat([6, n], 1, n, 1, p, 0)  # overwritten below with x_k = k + k i
    for part in (xs.re, xs.im):
        for k in range(n):
            v = k + 1
            e = v.bit_length()
            part.sign[0, k] = 0
            part.exp[0, k] = e
            part.mant[:, 0, k] = 0
            part.mant[L - 1, 0, k] = v << (64 - e)
    dx = mp.to_device(xs)
    out = {}
    mp.mpcg_set_stream()
    # warm-up of every kernel on a small case
    dW = mp.to_device(random_cmat([6, 16], 0, 16, 16, p, 2))
    wp = torch.zeros(16, dtype=torch.int32, device="cuda")
    mp.mp_zgetrf(16, dW, dW.ld, wp, 8, p, mp.MPCG_3M)
    for K in widths:
        log(f"full LU n={n} p={p} K={K}")
        dA = mp.to_device(A)
        dB = mp.device_empty(n, 1, p)
        mp.mp_cgemm(n, 1, n, dA, dA.ld, dx, dx.ld, dB, dB.ld, p)
        ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = mp.mp_zgetrf(n, dA, dA.ld, ipiv, K, p, mp.MPCG_3M)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mp.mp_zgetrs(n, 1, dA, dA.ld, ipiv, dB, dB.ld, p, mp.MPCG_3M)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if info != 0 or mp.mpcg_stream_status() != 0:
            raise RuntimeError(f"LU failed: info {info}, {mp.mpcg_last_error()}")
        h = mp.to_numpy(dB)
        err = Fraction(0)
        for k in range(n):
            comps = []
            for name in ("re", "im"):
                sg, ex, mt = h[name]
                if ex[0, k] == EXP_ZERO:
                    comps.append(Fraction(0))
                    continue
                M = 0
                for l in range(L - 1, -1, -1):
                    M = (M << 64) | int(mt[l, 0, k])
                v = Fraction(M) * Fraction(2) ** (int(ex[0, k]) - 64 * L)
                comps.append(-v if sg[0, k] else v)
            err = max(err, (abs(comps[0] - (k + 1)) + abs(comps[1] - (k + 1))) / (2 * (k + 1)))
        out[f"K{K}"] = {"getrf_s": t1 - t0, "getrs_s": t2 - t1, "max_rel_err": float(err)}
        log(f"  getrf {t1 - t0:.2f} s, getrs {t2 - t1:.2f} s, max relative error {float(err):.2e}")
        del dA, dB
    return out


def lu_update_stream():
    """The 31 trailing updates of a blocked LU of order 4096 with block 128
    (A22 := A22 - L21 U12, r x 128 times 128 x r, r = 3968 ... 128) at 256
    bits, in place through mp_cgemm_acc, planned from a spread bound and
    captured in one HIP graph that is replayed; the same stream of plain
    products C := L21 U12 is timed beside it."""
    import torch
    import paper_2307_06072_amd as mp
    from mpgen import random_cmat
    log("LU trailing-update stream: 31 in-place updates, graph-captured")
    p, b, N, R, bound = 256, 128, 4096, 2, 8
    sizes = [N - b * (j + 1) for j in range(N // b - 1)]
    ops = []
    for j, r in enumerate(sizes):
        A = mp.to_device(random_cmat([5, j], 0, r, b, p, R))
        B = mp.to_device(random_cmat([5, j], 1, b, r, p, R))
        C = mp.to_device(random_cmat([5, j], 2, r, r, p, R + 4))  # the trailing block A22
        ops.append((A, B, C))
    opt = mp.mpcg_options(mp.MPCG_SLICE_INT8, 0, 0, 0, bound)
    wsz = max(mp.mpcg_workspace_size(r, r, b, p, mp.MPCG_3M, mp.MPCG_EXACT, opt, bound) for r in sizes)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    work = sum(8.0 * r * r * b for r in sizes)
    out = {}
    mp.mpcg_set_workspace(ws.data_ptr(), wsz)
    try:
        def issue_acc():
            for (A, B, C) in ops:
                mp.mp_cgemm_acc(A.rows, B.cols, A.cols, A, A.ld, B, B.ld, C, C.ld, p, -1, mp.MPCG_3M,
                                mp.MPCG_EXACT, max_spread=bound)

        def issue_prod():
            for (A, B, C) in ops:
                mp.mp_cgemm_ex(A.rows, B.cols, A.cols, A, A.ld, B, B.ld, C, C.ld, p, mp.MPCG_3M, mp.MPCG_EXACT,
                               max_spread=bound)

        for name, issue in (("acc", issue_acc), ("prod", issue_prod)):
            mp.mpcg_set_stream()
            issue()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            issue()
            torch.cuda.synchronize()
            eager = time.perf_counter() - t0
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                    mp.mpcg_set_stream(side.cuda_stream)
                    issue()
            mp.mpcg_set_stream()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                g.replay()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            if mp.mpcg_stream_status() != 0:
                raise RuntimeError(mp.mpcg_last_error())
            out[name] = (dt, eager)
    finally:
        mp.mpcg_set_workspace(None, 0)
        mp.mpcg_set_stream()
    (dt, eager), (dtp, eagerp) = out["acc"], out["prod"]
    return {"lu_updates_n4096_b128_p256": {"form": "A22 := A22 - L21 U12 in place (mp_cgemm_acc)",
                                           "ms_per_replay": 1000 * dt, "8mnk_per_s": work / dt,
                                           "eager_ms": 1000 * eager, "products": len(sizes), "max_spread": bound,
                                           "plain_product_ms_per_replay": 1000 * dtp}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cgemm2048_p1024")
    ap.add_argument("--mode", default="3M", choices=["3M", "4M"])
    ap.add_argument("--scheme", default="exact", choices=["exact", "truncated"])
    ap.add_argument("--slice", default="int8", choices=["int8", "fp64"])
    ap.add_argument("--strassen", type=int, default=1, choices=[0, 1],
                    help="one level of Strassen's recursion over the slice products (same bits; INT8 exact)")
    ap.add_argument("--no-extras", action="store_true", help="skip the comparison family")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    ap.add_argument("--lu-widths", default="64,128,352",
                    help="block widths K of the paper-LU family (comma-separated)")
    ap.add_argument("--lu-precs", default="256",
                    help="precisions of the paper-LU family (comma-separated bits)")
    ap.add_argument("--family", choices=["batched", "lu", "codec", "lufull", "lupaper", "adaptive", "parts", "small",
                                         "f64"],
                    default=None,
                    help="only run one comparison family (for profiling) and print its record")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; --gpus must be 1 "
              "(the product shards by output blocks without any exchange, see the design notes)",
              file=sys.stderr)
        return 2

    import torch
    import paper_2307_06072_amd as mp
    from mpgen import workload_inputs

    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 3}))
        return 0
    if args.family:
        rec = {"batched": batched_case, "lu": lu_update_stream, "codec": codec_case,
               "lufull": lambda: lu_full_case(),
               "lupaper": lambda: lu_paper_case(tuple(int(v) for v in args.lu_widths.split(",")),
                                                tuple(int(v) for v in args.lu_precs.split(","))),
               "adaptive": lambda: adaptive_case(*workload_inputs("cgemm2048_p1024")[4:], 1024),
               "parts": parts_case, "small": small_latency_case, "f64": f64_case}[args.family]()
        print(json.dumps({"family": args.family, **rec}), flush=True)
        return 0
    log(f"generating {args.workload}")
    m, n, k, p, A, B = workload_inputs(args.workload)
    dA, dB = mp.to_device(A), mp.to_device(B)
    dC = mp.device_empty(m, n, p)
    torch.cuda.synchronize()
    mode, scheme, sl = _mode(args.mode), _scheme(args.scheme), _slice(args.slice)
    log(f"timing {args.steps} steps after {args.warmup} warmup ({args.slice} {args.mode} {args.scheme})")
    dt, info, stages = time_calls(dA, dB, dC, m, n, k, p, mode, scheme, sl, args.steps, args.warmup,
                                  strassen=args.strassen)
    launches = 7 if info["strassen"] else 1  # slice GEMM launches per call
    ms = 1000.0 * dt / args.steps
    value = 8.0 * m * n * k * args.steps / dt
    log(f"{ms:.3f} ms/step, {value:.4e} 8mnk/s; stages us {['%.1f' % s for s in stages]}")

    gemm_us = stages[2]
    if args.slice == "int8":
        achieved = info["algo_ops"] / (gemm_us * 1e-6) / 1e12
        peak, unit = PEAK_INT8_TOPS, "TOP/s"
    else:
        achieved = info["algo_ops"] / (gemm_us * 1e-6) / 1e12
        peak, unit = PEAK_FP64_TFLOPS, "TFLOP/s"
    src = os.path.join(ROOT, "paper_2307_06072_amd", "csrc", "gemm_i8.hip")
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": (traffic_record(src, "strassen1" if info["strassen"] else "plain")
                        if args.slice == "int8" else None),
            "kernel": ((f"gemm_i8_p_kernel<{info['block']}, {info['nprod']}> (one real product per workgroup; slice-pair GEMM + carry chain)"
                        if info["apart"] else "gemm_i8_kernel (slice-pair GEMM + carry chain)")
                       if args.slice == "int8" else "rocblas_dgemm + f64_accumulate_kernel"),
            "launches_per_step": launches,
            "algo_ops_per_launch": info["algo_ops"] / launches, "avg_launch_us": gemm_us / launches}
    # the same instruction's rate with no memory traffic, beside the published peak
    meas, probe_shape = mfma_probe(0 if args.slice == "int8" else 1)
    roof["measured_peak"] = meas
    roof["frac_of_measured"] = achieved / meas
    roof["measured_peak_probe"] = probe_shape
    log(f"matrix-core probe: {meas:.0f} {unit} measured, slice GEMM at {achieved / meas:.3f} of it")
    split_b, round_b = stage_bytes(m, n, k, p, info, args.mode == "3M", args.slice == "fp64")
    stage_report = {
        "scan_us": stages[0], "split_us": stages[1], "gemm_us": stages[2], "round_us": stages[3],
        "split_GBps": split_b / (stages[1] * 1e-6) / 1e9 if stages[1] > 0 else None,
        "round_GBps": round_b / (stages[3] * 1e-6) / 1e9 if stages[3] > 0 else None,
        "hbm_peak_GBps": PEAK_HBM_GBS,
        "note": "split/scan include the scan read-back synchronisation; bytes are algorithmic",
    }

    extra = {}
    if not args.no_extras:
        log("comparison family 512^3 at 512 bits")
        m2, n2, k2, p2, A2, B2 = workload_inputs("cgemm512_p512")
        dA2, dB2 = mp.to_device(A2), mp.to_device(B2)
        dC2 = mp.device_empty(m2, n2, p2)
        fam = {}
        for sl2, md2, sc2 in [("fp64", "4M", "exact"), ("int8", "4M", "exact"), ("int8", "3M", "exact"),
                              ("fp64", "4M", "truncated"), ("int8", "4M", "truncated"),
                              ("int8", "3M", "truncated")]:
            dt2, info2, st2 = time_calls(dA2, dB2, dC2, m2, n2, k2, p2, _mode(md2), _scheme(sc2), _slice(sl2),
                                         steps=5, warmup=1)
            key = f"{sl2}_{md2}_{sc2}"
            peak2 = PEAK_FP64_TFLOPS if sl2 == "fp64" else PEAK_INT8_TOPS
            fam[key] = {"ms_per_call": 1000 * dt2 / 5, "8mnk_per_s": 8.0 * m2 * n2 * k2 * 5 / dt2,
                        "gemm_us": st2[2], "gemm_frac_of_peak": info2["algo_ops"] / (st2[2] * 1e-6) / 1e12 / peak2,
                        "S_A": info2["S_A"], "cutoff": info2["cutoff"], "pairs": info2["pairs"]}
            log(f"  {key}: {fam[key]['ms_per_call']:.3f} ms")
        dt2, info2, st2 = time_calls(dA2, dB2, dC2, m2, n2, k2, p2, M3_MODE, 0, 0, steps=5, warmup=1, strassen=1)
        fam["int8_3M_exact_strassen"] = {"ms_per_call": 1000 * dt2 / 5, "8mnk_per_s": 8.0 * m2 * n2 * k2 * 5 / dt2,
                                         "gemm_us": st2[2], "strassen": info2["strassen"],
                                         "gemm_frac_of_peak": info2["algo_ops"] / (st2[2] * 1e-6) / 1e12 /
                                         PEAK_INT8_TOPS}
        log(f"  int8_3M_exact_strassen: {fam['int8_3M_exact_strassen']['ms_per_call']:.3f} ms")
        fam["speedup_int8_3m_over_fp64_4m_exact"] = fam["fp64_4M_exact"]["ms_per_call"] / fam["int8_3M_exact"]["ms_per_call"]
        # each form's slice products against its instruction's measured register-only rate
        meas8 = meas if args.slice == "int8" else mfma_probe(0)[0]
        meas64 = mfma_probe(1)[0]
        fam["measured_peak_int8_TOPs"] = meas8
        fam["measured_peak_fp64_TFLOPs"] = meas64
        for key2, rec2 in fam.items():
            if isinstance(rec2, dict) and "gemm_frac_of_peak" in rec2:
                pk2 = PEAK_FP64_TFLOPS if key2.startswith("fp64") else PEAK_INT8_TOPS
                ms2 = meas64 if key2.startswith("fp64") else meas8
                rec2["gemm_frac_of_measured"] = rec2["gemm_frac_of_peak"] * pk2 / ms2
        fam["speedup_int8_3m_over_fp64_4m_truncated"] = (fam["fp64_4M_truncated"]["ms_per_call"] /
                                                         fam["int8_3M_truncated"]["ms_per_call"])
        extra["cgemm512_p512"] = fam
        del dA2, dB2, dC2
        if args.workload == "cgemm2048_p1024" and args.scheme == "exact":
            other = 1 - args.strassen
            log(f"default workload, strassen={other}")
            dto, infoo, sto = time_calls(dA, dB, dC, m, n, k, p, mode, scheme, sl, steps=2, warmup=1, strassen=other)
            extra[f"cgemm2048_p1024_strassen{other}"] = {
                "ms_per_call": 1000 * dto / 2, "8mnk_per_s": 8.0 * m * n * k * 2 / dto, "strassen": infoo["strassen"],
                "stage_us": sto, "ksplit": infoo["ksplit"], "block": infoo["block"],
                "gemm_frac_of_peak": infoo["algo_ops"] / (sto[2] * 1e-6) / 1e12 / PEAK_INT8_TOPS}
            extra.update(adaptive_case(A, B, p))
            log("default workload, truncated scheme")
            dtt, infot, stt = time_calls(dA, dB, dC, m, n, k, p, mode, _scheme("truncated"), sl, steps=2, warmup=1)
            extra["cgemm2048_p1024_truncated"] = {"ms_per_call": 1000 * dtt / 2, "8mnk_per_s": 8.0 * m * n * k * 2 / dtt,
                                                  "cutoff": infot["cutoff"], "pairs": infot["pairs"],
                                                  "gemm_frac_of_peak": infot["algo_ops"] / (stt[2] * 1e-6) / 1e12 / PEAK_INT8_TOPS}

    if not args.no_extras and args.workload == "cgemm2048_p1024":
        del dA, dB, dC
        for variant in ("cgemm2048_p1024_rowcol60", "cgemm2048_p1024_contract60"):
            log(f"{variant}: generating and timing")
            mv, nv, kv, pv, Av, Bv = workload_inputs(variant)
            dAv, dBv = mp.to_device(Av), mp.to_device(Bv)
            dCv = mp.device_empty(mv, nv, pv)
            dtv, infov, stv = time_calls(dAv, dBv, dCv, mv, nv, kv, pv, mode, scheme, sl, steps=2, warmup=1,
                                         strassen=args.strassen)
            extra[variant] = {"ms_per_call": 1000 * dtv / 2, "8mnk_per_s": 8.0 * mv * nv * kv * 2 / dtv,
                              "S_A": infov["S_A"], "S_B": infov["S_B"], "pairs": infov["pairs"],
                              "strassen": infov["strassen"], "stage_us": stv,
                              "gemm_frac_of_peak": infov["algo_ops"] / (stv[2] * 1e-6) / 1e12 / PEAK_INT8_TOPS}
            del dAv, dBv, dCv, Av, Bv

    if not args.no_extras and args.workload == "cgemm2048_p1024":
        extra.update(parts_case())

    if not args.no_extras:
        extra.update(small_latency_case())
        extra.update(batched_case())
        extra.update(lu_update_stream())
        extra.update(lu_full_case())
        extra.update(codec_case())

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, B, m, n, k, p, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": value, "unit": "8mnk/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8" if args.slice == "int8" else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload} {args.slice.upper()}-{args.mode} {args.scheme}", "m": m, "n": n,
                   "k": k, "prec_bits": p, "mode": args.mode, "scheme": args.scheme, "slice": args.slice,
                   "S_A": info["S_A"], "S_B": info["S_B"], "cutoff": info["cutoff"], "pairs": info["pairs"],
                   "ksplit": info["ksplit"], "block": info["block"], "strassen_levels": info["strassen"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages": stage_report,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
