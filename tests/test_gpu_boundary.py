"""The decode entry point with an argument struct and flags (early stop off,
validation posteriors, asynchronous enqueueing), several rounds from an
imported state, a pool sized from an HBM budget and the chunk tuning keys,
through the C-ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sp import decode as odecode, run_rounds as orun_rounds  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from tests._msg import TOL_FP32, fourier, from_state, to_state  # noqa: E402
from tests.test_gpu_parity import CASES, _dev, _setup  # noqa: E402

pytestmark = pytest.mark.gpu


def _np(r):
    return {k: v.cpu().numpy() for k, v in r.items()}


@pytest.mark.parametrize("mode,prec", [("fused", "fp32"), ("fused", "fp16"), ("plain", "fp32")])
def test_decode_ex_without_flags_and_async_equal_decode(mode, prec):
    """decode_ex with no flags, and with ASYNC (every round enqueued, no host
    read of the active count), give exactly ldpc_fd_decode's outputs."""
    name, m, k, N, F, ebn0 = CASES[5]
    print(f"[case] decode_ex {mode} {prec}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    dec = D.Decoder(gcode, F, prec, mode)
    ref = _np(dec(L, 30))
    for flags in (0, D.FLAG_ASYNC):
        got = _np(dec.decode_ex(L, 30, flags))
        for key in ref:
            assert np.array_equal(got[key], ref[key]), (flags, key)
    gcode.close()


@pytest.mark.parametrize("mode", ["fused", "plain"])
def test_no_early_stop_runs_every_round_like_the_oracle(mode):
    """NO_EARLY_STOP: every frame runs max_iter rounds; the last round's
    decisions equal the oracle's decode without stopping (except at near-ties)
    and the converged bit is that round's codeword test."""
    name, m, k, N, F, ebn0 = CASES[0]
    print(f"[case] no early stop {mode}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    dec = D.Decoder(gcode, F, "fp32", mode)
    out = _np(dec.decode_ex(_dev(llr), 12, D.FLAG_NO_EARLY_STOP))
    ref = odecode(tc, llr.astype(np.float64), 12, early_stop=False)
    assert np.all(out["iters"] == 12)
    same = np.all(out["hard"] == ref.hard, axis=1)
    assert same.mean() >= 0.97, same.mean()
    conv = (out["status"] & D.STATUS_CONVERGED) != 0
    assert np.array_equal(conv[same], ref.converged[same])
    assert np.array_equal(out["synd"].astype(np.int64), enc.syndrome(out["hard"].astype(np.int64)))
    gcode.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_validation_flag_writes_the_stopping_round_posterior(prec):
    name, m, k, N, F, ebn0 = CASES[5]
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    dec = D.Decoder(gcode, F, prec, "fused")
    out = dec.decode_ex(L, 20, D.FLAG_VALIDATION)
    post = out["posterior"].cpu().numpy()
    assert np.array_equal(post, dec.posterior().cpu().numpy())
    assert np.allclose(post.sum(-1), 1.0, atol=1e-12)
    gcode.close()


def test_decode_ex_rejects_bad_flags():
    name, m, k, N, F, ebn0 = CASES[0]
    code, enc, cw, llr, tc = _setup(m, k, N, 4, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    with pytest.raises(D.LdpcFdError) as ei:
        D.Decoder(gcode, 4, "fp32", "fused").decode_ex(L, 10, 8)
    assert ei.value.rc == D.E_INVALID
    with pytest.raises(D.LdpcFdError) as ei:
        D.Decoder(gcode, 4, "fp32", "logsp").decode_ex(L, 10, D.FLAG_ASYNC)
    assert ei.value.rc == D.E_UNSUPPORTED
    with pytest.raises(D.LdpcFdError) as ei:
        D.Decoder(gcode, 4, "fp32", "plain").decode_ex(L, 10, D.FLAG_VALIDATION)
    assert ei.value.rc == D.E_UNSUPPORTED
    gcode.close()


@pytest.mark.parametrize("mode,prec", [("fused", "fp32"), ("plain", "fp32"), ("fused", "fp16")])
def test_run_rounds_chains_single_rounds(mode, prec):
    """run_rounds(3) from the channel equals three chained single rounds, and
    (FP32) the oracle's third round within the FP32 message tolerance."""
    name, m, k, N, F, ebn0 = CASES[2]
    print(f"[case] run_rounds {mode} {prec}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    st = None
    for _ in range(3):
        r = D.round_step(gcode, L, st, mode, prec)
        st = r["c2v"]
    multi = D.run_rounds(gcode, L, 3, None, mode, prec)
    torch.cuda.synchronize()
    assert torch.equal(multi["c2v"], st)
    for key in ("hard", "fsynd", "synd"):
        assert torch.equal(multi[key], r[key]), key
    # from an imported state: one more round
    more = D.run_rounds(gcode, L, 1, st, mode, prec)
    one = D.round_step(gcode, L, st, mode, prec)
    assert torch.equal(more["c2v"], one["c2v"])
    if prec == "fp32":
        c2vs, _, _ = orun_rounds(tc, llr.astype(np.float64), 3)
        err = np.abs(from_state(multi["c2v"].cpu().numpy()) - fourier(c2vs[2])).max()
        assert err < 3 * TOL_FP32, err
    gcode.close()


def test_pool_sized_from_a_budget():
    specs = [CASES[2], CASES[5]]
    codes = []
    for name, m, k, N, F, ebn0 in specs:
        code, enc, cw, llr, tc = _setup(m, k, N, 4, ebn0)
        codes.append(D.Code.from_synth(code))
    budget = 3 << 20
    pool = D.Pool(codes, None, "fp16", hbm_budget=budget)
    for k, c in enumerate(codes):
        assert pool.slots[k] == (budget // 2) // D.pool_slot_bytes(c, "fp16")
    assert pool.slots == D.pool_budget_slots(codes, budget, "fp16")
    # the query checks its arguments like the pool it sizes
    with pytest.raises(D.LdpcFdError) as ei:
        D.pool_budget_slots(codes, 1000, "fp32")
    assert ei.value.rc == D.E_NOMEM
    with pytest.raises(D.LdpcFdError) as ei:
        D.pool_budget_slots(codes, 0, "fp16")
    assert ei.value.rc == D.E_INVALID
    with pytest.raises(D.LdpcFdError) as ei:
        D.pool_budget_slots(codes, budget, "log8")
    assert ei.value.rc == D.E_INVALID
    pool.close()
    with pytest.raises(D.LdpcFdError) as ei:
        D.Pool(codes, None, "fp32", hbm_budget=1000)
    assert ei.value.rc == D.E_NOMEM
    for c in codes:
        c.close()


def test_chunk_tuning_keys_round_trip_and_reject_out_of_range_values():
    """FIRST_CHUNK, TAIL_CHUNK and BATCH_RETIRE read back what was set (0 is
    each one's default) and refuse values outside their ranges with
    E_INVALID, leaving the setting unchanged."""
    name, m, k, N, F, ebn0 = CASES[0]
    code, enc, cw, llr, tc = _setup(m, k, N, 4, ebn0)
    gcode = D.Code.from_synth(code)
    t = gcode.get_tuning()
    assert (t["first_chunk"], t["tail_chunk"], t["batch_retire"]) == (0, 0, 0)
    gcode.set_tuning(first_chunk=9, tail_chunk=17, batch_retire=1)
    t = gcode.get_tuning()
    assert (t["first_chunk"], t["tail_chunk"], t["batch_retire"]) == (9, 17, 1)
    for key, bad in (("first_chunk", -1), ("first_chunk", 1001), ("tail_chunk", 1001), ("batch_retire", 2)):
        with pytest.raises(D.LdpcFdError) as ei:
            gcode.set_tuning(**{key: bad})
        assert ei.value.rc == D.E_INVALID, key
    t = gcode.get_tuning()
    assert (t["first_chunk"], t["tail_chunk"], t["batch_retire"]) == (9, 17, 1)
    gcode.close()
