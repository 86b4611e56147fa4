"""Serving loop: Poisson arrivals of requests over several codes, admission by
HBM footprint, continuous batching, latency percentiles.  Every admitted frame
comes back exactly once with the result it has when decoded alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1008_4370_amd import decoder as D  # noqa: E402
from paper_1008_4370_amd import serving  # noqa: E402

pytestmark = pytest.mark.gpu


def test_serving_loop_returns_every_frame_once():
    specs = [(4, 4, 128), (6, 6, 60), (8, 16, 32)]
    banks = serving.make_banks(specs, snr_range=(2.5, 3.5), snr_points=2, frames_per_point=64, seed=77)
    # footprint admission: a budget that holds only a few slots per code
    budget = 3 * 40 * max(D.pool_slot_bytes(b.gcode, "fp16") for b in banks)
    slots = serving.slots_for_budget(banks, budget, "fp16")
    assert all(s >= 40 for s in slots)
    r = serving.serve(banks, offered_fps=20000, duration_s=0.5, prec="fp16", max_iter=30, request_frames=8,
                      hbm_budget=budget, warmup_s=0.0, record=True)
    assert r["frames"] > 0 and r["slots"] == slots
    assert r["frame_latency_ms"]["p50"] <= r["frame_latency_ms"]["p99"]
    # each frame decoded in the mix equals the same frame decoded alone
    rec = r["records"]
    for k, b in enumerate(banks):
        mine = [x for x in rec if x[0] == k]
        assert mine
        for p in range(len(b.ebn0)):
            idx = [x for x in mine if x[1] == p]
            if not idx:
                continue
            alone = D.decode(b.gcode, b.llr[p].contiguous(), 30, prec="fp16", mode="fused")
            it = alone["iters"].cpu().numpy()
            hd = alone["hard"].cpu().numpy()
            for (_, _, f, iters, hard) in idx:
                assert iters == it[f] and np.array_equal(hard, hd[f]), (k, p, f)
    for b in banks:
        b.gcode.close()
