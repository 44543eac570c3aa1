"""The matrix-core rate probe behind the benchmark's measured peak: both
instructions run, and their rates lie between a fifth of MI355X's published
dense peak and 10% above it (5.0 POP/s INT8, 78.6 TFLOP/s FP64)."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,peak", [(0, 5000.0), (1, 78.6)])
def test_probe_rate_is_plausible(kind, peak):
    import torch
    import paper_2307_06072_amd as mp
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    mp.mpcg_set_stream()
    blocks, iters = 256 * 8, 64
    ops, ms = mp.mpcg_probe_mfma(kind, blocks, iters, sink.data_ptr())
    assert ops == blocks * 4 * iters * 8 * (32768 if kind == 0 else 2048)
    ops, ms = mp.mpcg_probe_mfma(kind, blocks, iters, sink.data_ptr())
    rate = ops / (ms * 1e-3) / 1e12
    print(f"kind {kind}: {rate:.1f} per {ms:.3f} ms", flush=True)
    assert peak / 5 < rate < 1.1 * peak, rate
