"""GPU parity of the conventional log-domain SP decoder (LDPC_FD_MODE_LOGSP, the
Log-SP of Sec. 2.2 that Table 1 compares against) with the FP64 oracle: the
oracle's messages are probability-domain pmfs, the decoder's are log2 pmfs
with maximum 0, so the comparison takes both to normalised linear pmfs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sp import TannerCode, channel_prior, decode as odecode, run_rounds  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from paper_1008_4370_amd import synth  # noqa: E402
from tests._msg import fsynd_near_tie, near_tie_bits  # noqa: E402
from tests.test_gpu_parity import CASES, _check_outputs, _dev, _full_run, _setup  # noqa: E402

pytestmark = pytest.mark.gpu

FLOOR = 200.0
# Normalised linear pmfs: absolute difference.  FP32 log-sum-exp on log values
# of magnitude <= 200 carries ~1e-5 absolute error in the log, i.e. ~1e-5
# relative on every entry.
TOL_PMF = 1e-4
# log2 entries of probability above 2^-20 (relative to the largest entry):
# absolute difference in log2 units.
TOL_LOG = 2e-3


def to_log(p: np.ndarray) -> np.ndarray:
    """Prob-domain messages -> log2 pmfs with maximum 0, floored."""
    with np.errstate(divide="ignore"):
        lg = np.log2(p)
    lg = lg - lg.max(-1, keepdims=True)
    return np.maximum(lg, -FLOOR).astype(np.float32)


def to_pmf(lg: np.ndarray) -> np.ndarray:
    p = np.exp2(np.asarray(lg, dtype=np.float64))
    return p / p.sum(-1, keepdims=True)


def _compare(got_log: np.ndarray, want_p: np.ndarray):
    got = to_pmf(got_log)
    want = want_p / want_p.sum(-1, keepdims=True)
    err_p = np.abs(got - want).max()
    wl = to_log(want)
    big = wl > -20
    err_l = np.abs(np.asarray(got_log, np.float64) - wl)[big].max()
    assert np.all(np.asarray(got_log) <= 0) and np.all(np.asarray(got_log) >= -FLOOR)
    assert np.all(np.asarray(got_log).max(-1) == 0)
    return err_p, err_l


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_logsp_one_round_message_parity(case):
    """From the same imported state, one Log-SP round matches the oracle's round
    (messages within TOL_PMF as pmfs and TOL_LOG in log2 on entries above
    2^-20), decisions equal except near-ties, direct syndromes bit-exact."""
    name, m, k, N, F, ebn0 = case
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    print(f"[case] {name} logsp F={F}", flush=True)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    c2vs, v2cs, decs = run_rounds(tc, llr.astype(np.float64), 3)
    out = D.round_step(gcode, L, None, "logsp")
    torch.cuda.synchronize()
    p0 = channel_prior(llr.astype(np.float64), m)[:, tc.edge_var]
    ep, el = _compare(out["v2c"].cpu().numpy(), p0)
    assert ep < TOL_PMF and el < TOL_LOG, (ep, el)
    ep, el = _compare(out["c2v"].cpu().numpy(), c2vs[0])
    assert ep < TOL_PMF and el < TOL_LOG, (ep, el)
    for i in (0, 1):
        out = D.round_step(gcode, L, _dev(to_log(c2vs[i])), "logsp")
        torch.cuda.synchronize()
        ep, el = _compare(out["v2c"].cpu().numpy(), v2cs[i])
        assert ep < TOL_PMF and el < TOL_LOG, ("v2c", i, ep, el)
        ep, el = _compare(out["c2v"].cpu().numpy(), c2vs[i + 1])
        assert ep < TOL_PMF and el < TOL_LOG, ("c2v", i, ep, el)
        hard = out["hard"].cpu().numpy()
        d = decs[i]
        ok = near_tie_bits(d.qbits)
        assert np.array_equal(hard[~ok], d.hard[~ok])
        assert np.array_equal(out["synd"].cpu().numpy().astype(np.int64), enc.syndrome(hard.astype(np.int64)))
        fs_ok = fsynd_near_tie(tc, d.post)
        fs = out["fsynd"].cpu().numpy()
        assert np.array_equal(fs[~fs_ok], d.fsynd[~fs_ok])
    gcode.close()


def test_logsp_full_run_parity_gf4_n96_1000_frames():
    b = synth.make_batch("gf4_n96")
    tc = TannerCode(b.code.M, b.code.N, b.code.m, b.code.row_ptr, b.code.col, b.code.val, b.code.poly)
    print("[case] gf4_n96 full logsp", flush=True)
    ref = odecode(tc, b.llr, 50)
    out = _full_run(b.code, b.llr, 50, "fp32", "logsp")
    conv = _check_outputs(out, b.enc, 50)
    same = (np.all(out["hard"] == ref.hard, axis=1) & (out["iters"] == ref.iters) & (conv == ref.converged))
    assert same.mean() >= 0.99, same.mean()


def test_logsp_gf64_n1000_sampled_parity_and_agreement_with_lfsp():
    """GF(64) (2,6) N=1000 at 2.5 dB, 512 frames: outputs self-consistent, a
    sample of frames identical to the oracle's decode, and per-frame results
    equal to the Log-Fourier decoder's on all but near-tie trajectories."""
    b = synth.make_batch("gf64_n1000", point=2, frames=512)
    print("[case] gf64_n1000 logsp 512 frames", flush=True)
    out = _full_run(b.code, b.llr, 100, "fp32", "logsp")
    conv = _check_outputs(out, b.enc, 100)
    assert conv.mean() > 0.9
    idx = np.arange(0, 512, 128)
    tc = TannerCode(b.code.M, b.code.N, b.code.m, b.code.row_ptr, b.code.col, b.code.val, b.code.poly)
    ref = odecode(tc, b.llr[idx], 100)
    assert np.all(np.all(out["hard"][idx] == ref.hard, axis=1))
    assert np.array_equal(out["iters"][idx], ref.iters)
    lf = _full_run(b.code, b.llr, 100, "fp32", "fused")
    same = np.all(out["hard"] == lf["hard"], axis=1) & (out["iters"] == lf["iters"])
    print(f"[logsp vs lfsp] same {same.mean():.4f}", flush=True)
    assert same.mean() >= 0.98


def test_logsp_edge_cases():
    b = synth.make_batch("gf4_n96", frames=5)
    gcode = D.Code.from_synth(b.code)
    z = torch.zeros((5, b.code.N, b.code.m), dtype=torch.float32, device="cuda")
    r = D.decode(gcode, z, 10, mode="logsp")
    assert int(r["hard"].max()) == 0 and bool((r["iters"] == 1).all())
    r = D.decode(gcode, _dev(b.llr), 1, mode="logsp")
    assert bool((r["iters"] == 1).all())
    # FP32 storage only
    with pytest.raises(D.LdpcFdError) as ei:
        D.workspace_bytes(gcode, 5, "fp16", "logsp")
    assert ei.value.rc == D.E_UNSUPPORTED
    gcode.close()


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[5], CASES[7], CASES[8]], ids=lambda c: c[0])
def test_logsp_8bit_storage_equals_the_emulated_8bit_grid(case):
    """LDPC_FD_LOG8: messages stored as one byte (code k of the log2
    probability -k).  The decode is identical, frame by frame, to FP32
    storage with every stored message rounded onto the same grid in place
    (QUANT_BITS = 8, QUANT_STEP = 4096: step 1), and the workspace holds a
    quarter of the message bytes."""
    name, m, k, N, F, ebn0 = case
    print(f"[case] logsp 8-bit {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    r8 = {k2: v.cpu().numpy() for k2, v in D.decode(gcode, L, 30, prec="log8", mode="logsp").items()}
    gcode.set_tuning(quant_bits=8, quant_step=4096)
    rq = {k2: v.cpu().numpy() for k2, v in D.decode(gcode, L, 30, prec="fp32", mode="logsp").items()}
    gcode.set_tuning(quant_bits=0)
    for key in ("hard", "synd", "iters", "status"):
        assert np.array_equal(r8[key], rq[key]), key
    _check_outputs(r8, enc, 30)
    w8 = D.workspace_bytes(gcode, F, "log8", "logsp")
    w32 = D.workspace_bytes(gcode, F, "fp32", "logsp")
    msg = F * code.E * code.q
    assert w32 - w8 >= 2 * (3 * msg) - 2 * 512, (w32, w8)
    gcode.close()


def test_logsp_8bit_storage_gf64_n1000_fer():
    """GF(64) (2,6) N=1000, 2048 frames at 2.5 dB: 8-bit Log-SP messages keep
    the FP32 Log-SP frame error rate (the log domain holds its FER down to
    5-bit messages), and LOG8 is rejected outside the LOGSP mode."""
    b = synth.make_batch("gf64_n1000", point=2, frames=2048)
    print("[case] gf64_n1000 logsp 8-bit 2048 frames", flush=True)
    o32 = _full_run(b.code, b.llr, 100, "fp32", "logsp")
    o8 = _full_run(b.code, b.llr, 100, "log8", "logsp")
    c8 = _check_outputs(o8, b.enc, 100)
    fer32 = np.any(o32["hard"] != b.cw, axis=1).mean()
    fer8 = np.any(o8["hard"] != b.cw, axis=1).mean()
    print(f"[logsp 8-bit] FER fp32 {fer32:.2e} log8 {fer8:.2e}", flush=True)
    assert fer8 <= fer32 + 3.0 / 2048
    assert c8.mean() > 0.99
    gcode = D.Code.from_synth(b.code)
    for mode in ("fused", "plain", "fsp"):
        with pytest.raises(D.LdpcFdError) as ei:
            D.workspace_bytes(gcode, 16, "log8", mode)
        assert ei.value.rc == D.E_UNSUPPORTED
    # one round from an imported state is an FP32 operation
    with pytest.raises(D.LdpcFdError) as ei:
        D.round_step(gcode, _dev(b.llr[:4]), None, "logsp", "log8")
    assert ei.value.rc == D.E_UNSUPPORTED
    gcode.close()
