"""Synthetic input generators: graph structure, encoder and channel statistics."""
import numpy as np
import pytest

from paper_1008_4370_amd import synth


@pytest.mark.parametrize("N,k,m,degs", [(1000, 6, 6, {6: 331, 7: 2}), (512, 6, 6, {6: 169, 5: 2}),
                                        (96, 4, 2, {4: 48}), (512, 8, 8, {8: 128}),
                                        (256, 16, 8, {16: 32})])
def test_configuration_model(N, k, m, degs):
    c = synth.make_code(N, k, m)
    d = np.diff(c.row_ptr)
    assert dict(zip(*np.unique(d, return_counts=True))) == degs
    assert np.all(np.bincount(c.col, minlength=N) == 2)          # column weight 2
    key = np.repeat(np.arange(c.M), d).astype(np.int64) * N + c.col
    assert len(np.unique(key)) == len(key)                        # no double edges
    assert np.all((c.val >= 1) & (c.val < (1 << m)))
    c2 = synth.make_code(N, k, m)
    assert np.array_equal(c.col, c2.col) and np.array_equal(c.val, c2.val)


@pytest.mark.parametrize("name", ["gf4_n96", "gf16_n2048"])
def test_encoder_produces_codewords(name):
    w = synth.WORKLOADS[name]
    code = synth.make_code(w["N"], w["k"], w["m"])
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, 20)
    assert np.all(enc.syndrome(cw) == 0)
    assert enc.K == code.N - enc.rank
    assert np.any(cw != 0)


def test_channel_llr_statistics():
    code = synth.make_code(96, 4, 2)
    enc = synth.Encoder(code)
    cw = np.zeros((2000, code.N), dtype=np.int64)
    L = synth.bpsk_awgn_llr(cw, 2, 2.0, code.design_rate, seed=1)
    s2 = synth.sigma2_from_ebn0(2.0, code.design_rate)
    assert abs(L.mean() - 2 / s2) < 0.02 * (2 / s2)
    assert abs(L.var() - 4 / s2) < 0.03 * (4 / s2)


def test_irregular_column_weights():
    """Column weights follow the requested fractions (rounding absorbed by the
    largest), rows stay near-regular, no double edges, codewords exist."""
    vd = synth.irregular_var_degrees(1000, {2: 0.7, 3: 0.2, 4: 0.1}, seed=3)
    assert dict(zip(*np.unique(vd, return_counts=True))) == {2: 700, 3: 200, 4: 100}
    c = synth.make_code(1000, 6, 6, var_degrees=vd)
    assert np.array_equal(np.bincount(c.col, minlength=1000), vd)
    d = np.diff(c.row_ptr)
    assert c.M == round(vd.sum() / 6) and d.max() - d.min() <= 1 and d.sum() == vd.sum()
    key = np.repeat(np.arange(c.M), d).astype(np.int64) * 1000 + c.col
    assert len(np.unique(key)) == len(key)
    vd1 = synth.irregular_var_degrees(64, {1: 0.05, 2: 0.6, 3: 0.25, 5: 0.1}, seed=44)
    c1 = synth.make_code(64, 5, 4, var_degrees=vd1)
    enc = synth.Encoder(c1)
    assert np.all(enc.syndrome(synth.random_codewords(enc, 10)) == 0)


def test_irregular_workload_batch():
    b = synth.make_batch("gf64_n1000_irr", frames=4)
    assert b.code.M == 400 and np.all(b.enc.syndrome(b.cw) == 0)
    assert sorted(set(np.bincount(b.code.col, minlength=b.code.N))) == [2, 3, 4]
