"""Autotuner bookkeeping (host only): table keys, lane-entry choices, and the
committed table's entries are launch choices the library accepts."""
import json
import os

from paper_1008_4370_amd import autotune


class _FakeCode:
    def __init__(self, m, kmax, N, E):
        self.m, self.kmax, self.N, self.E = m, kmax, N, E


def test_frames_bucket():
    assert [autotune.frames_bucket(F) for F in (1, 2, 3, 4096, 4097, 6000)] == [1, 2, 4, 4096, 8192, 8192]


def test_key_and_lane_choices():
    assert autotune.key(_FakeCode(6, 7, 1000, 2000), "fp32", 4096) == "m6_k7_N1000_E2000_fp32_F4096"
    assert autotune.lane_choices(2, 4) == [4]
    assert autotune.lane_choices(3, 4) == [4, 8]
    assert autotune.lane_choices(6, 7) == [4, 8, 16]
    assert autotune.lane_choices(8, 8) == [4, 8, 16]
    assert autotune.lane_choices(8, 16) == [4, 8]
    assert autotune.lane_choices(2, 16) == [4]


def test_committed_table_is_valid():
    if not os.path.exists(autotune.TABLE):
        return
    with open(autotune.TABLE) as fh:
        table = json.load(fh)
    for k, ent in table.items():
        m = int(k.split("_")[0][1:])
        kmax = int(k.split("_")[1][1:])
        assert ent["lane_entries"] in autotune.lane_choices(m, kmax), k
        assert ent["grid_blocks"] % 8 == 0 and 8 <= ent["grid_blocks"] <= 1 << 20, k
        assert 1 <= ent["chunk"] <= 64, k
        if "tail_entries" in ent:
            assert ent["tail_entries"] in autotune.lane_choices(m, kmax), k
            assert ent["tail_frames"] >= 0, k
        assert ent["ms"] <= ent["default_ms"] * 1.05, k


def test_fer_helpers():
    from paper_1008_4370_amd import fer
    lo, hi = fer.wilson(10, 1000)
    assert lo < 0.01 < hi and 0.004 < lo and hi < 0.02
    a = [{"ebn0": 2.0, "fer": 1e-1}, {"ebn0": 2.5, "fer": 1e-3}]
    b = [{"ebn0": 2.0, "fer": 1e-1}, {"ebn0": 3.0, "fer": 1e-3}]
    assert abs(fer.crossing_db(a, 1e-2) - 2.25) < 1e-12
    assert abs(fer.gap_db(a, b, 1e-2) - 0.25) < 1e-12
    assert fer.crossing_db(a, 1e-4) is None
