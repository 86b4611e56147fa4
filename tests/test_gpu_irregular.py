"""GPU parity for codes whose column weights are not all 2 (the extension to
irregular codes of Sec. 2): the PLAIN decoder's general variable node (the
j-fold log-convolution of Sec. 3.2 through the convolution theorem) and the
Log-SP decoder, both against the FP64 oracle, which takes any column weights."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sp import TannerCode, channel_prior, decode as odecode, run_rounds  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from paper_1008_4370_amd import synth  # noqa: E402
from tests._msg import TOL_FP32, fourier, from_state, fsynd_near_tie, near_tie_bits, to_state  # noqa: E402
from tests.test_gpu_logsp import TOL_LOG, TOL_PMF, _compare, to_log  # noqa: E402
from tests.test_gpu_parity import _check_outputs, _dev  # noqa: E402

pytestmark = pytest.mark.gpu

# (name, m, k, N, frames, Eb/N0, {column weight: fraction}); weight-1 columns
# have no extrinsic input at the variable node; weight 5..6 stress the j-fold
# products.
CASES = [
    ("gf4_irr", 2, 4, 96, 37, 2.0, {2: 0.6, 3: 0.3, 4: 0.1}),
    ("gf16_irr_w1", 4, 5, 64, 29, 2.5, {1: 0.05, 2: 0.6, 3: 0.25, 5: 0.1}),
    ("gf64_irr", 6, 6, 60, 21, 2.5, {2: 0.7, 3: 0.2, 4: 0.1}),
    ("gf256_irr", 8, 8, 32, 7, 3.0, {2: 0.5, 3: 0.3, 6: 0.2}),
]


def _setup(case, seed=0):
    name, m, k, N, F, ebn0, dist = case
    vd = synth.irregular_var_degrees(N, dist, seed=40 + m + seed)
    code = synth.make_code(N, k, m, seed_graph=700 + m + seed, seed_labels=750 + k + seed, var_degrees=vd)
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, F, seed=15 + seed)
    llr = synth.bpsk_awgn_llr(cw, m, ebn0, code.design_rate, seed=16 + seed)
    tc = TannerCode(code.M, code.N, code.m, code.row_ptr, code.col, code.val, code.poly)
    return code, enc, cw, llr, tc


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_irregular_plain_one_round_message_parity(case):
    """One PLAIN round from the oracle's state: messages within 1e-4 in the
    linear Fourier domain, decisions equal except near-ties, direct syndromes
    bit-exact for the GPU's decisions, and the FP64 posterior of the imported
    state equal to the oracle's."""
    code, enc, cw, llr, tc = _setup(case)
    print(f"[case] {case[0]} plain irregular F={len(llr)}", flush=True)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    c2vs, v2cs, decs = run_rounds(tc, llr.astype(np.float64), 3)
    out = D.round_step(gcode, L, None, "plain")
    torch.cuda.synchronize()
    p0 = channel_prior(llr.astype(np.float64), case[1])[:, tc.edge_var]
    assert np.abs(from_state(out["v2c"].cpu().numpy()) - fourier(p0)).max() < TOL_FP32
    assert np.abs(from_state(out["c2v"].cpu().numpy()) - fourier(c2vs[0])).max() < TOL_FP32
    for i in (0, 1):
        st = _dev(to_state(c2vs[i]))
        out = D.round_step(gcode, L, st, "plain")
        torch.cuda.synchronize()
        err_v = np.abs(from_state(out["v2c"].cpu().numpy()) - fourier(v2cs[i])).max()
        err_c = np.abs(from_state(out["c2v"].cpu().numpy()) - fourier(c2vs[i + 1])).max()
        assert err_v < TOL_FP32 and err_c < TOL_FP32, (i, err_v, err_c)
        d = decs[i]
        hard = out["hard"].cpu().numpy()
        ok = near_tie_bits(d.qbits)
        assert np.array_equal(hard[~ok], d.hard[~ok])
        assert np.array_equal(out["synd"].cpu().numpy().astype(np.int64), enc.syndrome(hard.astype(np.int64)))
        fs_ok = fsynd_near_tie(tc, d.post)
        assert np.array_equal(out["fsynd"].cpu().numpy()[~fs_ok], d.fsynd[~fs_ok])
        post = D.posterior(gcode, L, st).cpu().numpy()
        assert np.abs(post - d.post).max() < 1e-4
    gcode.close()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_irregular_logsp_one_round_message_parity(case):
    code, enc, cw, llr, tc = _setup(case)
    print(f"[case] {case[0]} logsp irregular F={len(llr)}", flush=True)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    c2vs, v2cs, decs = run_rounds(tc, llr.astype(np.float64), 3)
    for i in (0, 1):
        out = D.round_step(gcode, L, _dev(to_log(c2vs[i])), "logsp")
        torch.cuda.synchronize()
        ep, el = _compare(out["v2c"].cpu().numpy(), v2cs[i])
        assert ep < TOL_PMF and el < TOL_LOG, ("v2c", i, ep, el)
        ep, el = _compare(out["c2v"].cpu().numpy(), c2vs[i + 1])
        assert ep < TOL_PMF and el < TOL_LOG, ("c2v", i, ep, el)
        d = decs[i]
        hard = out["hard"].cpu().numpy()
        ok = near_tie_bits(d.qbits)
        assert np.array_equal(hard[~ok], d.hard[~ok])
        assert np.array_equal(out["synd"].cpu().numpy().astype(np.int64), enc.syndrome(hard.astype(np.int64)))
    gcode.close()


@pytest.mark.parametrize("mode", ["plain", "logsp"])
def test_irregular_full_decode_parity(mode):
    """GF(16) irregular code, 400 frames at 2.5 dB, max 50 rounds: per-frame
    results equal to the oracle's on all but near-tie trajectories."""
    case = ("gf16_irr_full", 4, 5, 120, 400, 2.5, {2: 0.7, 3: 0.2, 4: 0.1})
    code, enc, cw, llr, tc = _setup(case, seed=3)
    print(f"[case] gf16 irregular full {mode}", flush=True)
    ref = odecode(tc, llr, 50)
    gcode = D.Code.from_synth(code)
    r = D.decode(gcode, _dev(llr), 50, mode=mode)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items()}
    gcode.close()
    conv = _check_outputs(out, enc, 50)
    same = np.all(out["hard"] == ref.hard, axis=1) & (out["iters"] == ref.iters) & (conv == ref.converged)
    print(f"[irregular {mode}] same {same.mean():.4f} converged {conv.mean():.3f}", flush=True)
    assert same.mean() >= 0.99, same.mean()


def test_irregular_gf64_n1000_sampled_parity():
    """The 2048-frame GF(64) N=1000 irregular workload (weights 2/3/4) at 2.5 dB:
    outputs self-consistent, a frame sample identical to the oracle, PLAIN and
    LOGSP agreeing on all but near-tie trajectories."""
    b = synth.make_batch("gf64_n1000_irr", point=1)
    print("[case] gf64_n1000_irr plain + logsp", flush=True)
    gcode = D.Code.from_synth(b.code)
    L = _dev(b.llr)
    outs = {}
    for mode in ("plain", "logsp"):
        r = D.decode(gcode, L, 100, mode=mode)
        torch.cuda.synchronize()
        outs[mode] = {k: v.cpu().numpy() for k, v in r.items()}
        conv = _check_outputs(outs[mode], b.enc, 100)
        fer = np.any(outs[mode]["hard"] != b.cw, axis=1).mean()
        print(f"[irregular] {mode}: converged {conv.mean():.4f} FER {fer:.4f}", flush=True)
        assert conv.mean() > 0.9
    gcode.close()
    idx = np.arange(0, 2048, 512)
    tc = TannerCode(b.code.M, b.code.N, b.code.m, b.code.row_ptr, b.code.col, b.code.val, b.code.poly)
    ref = odecode(tc, b.llr[idx], 100)
    for mode in ("plain", "logsp"):
        assert np.all(np.all(outs[mode]["hard"][idx] == ref.hard, axis=1)), mode
        assert np.array_equal(outs[mode]["iters"][idx], ref.iters), mode
    same = np.all(outs["plain"]["hard"] == outs["logsp"]["hard"], axis=1)
    assert same.mean() >= 0.98, same.mean()


def test_irregular_codes_rejected_where_column_weight_2_is_needed():
    code, enc, cw, llr, tc = _setup(CASES[1])
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    for call in (lambda: D.decode(gcode, L, 10, mode="fused"),
                 lambda: D.round_step(gcode, L, None, "fused"),
                 lambda: D.Pool([gcode], [16], "fp32")):
        with pytest.raises(D.LdpcFdError) as ei:
            call()
        assert ei.value.rc == D.E_UNSUPPORTED
    gcode.close()
