"""Validation mode: FP64 symbol posteriors on the GPU against the FP64 oracle's
tentative-decision posteriors (Sec. 2.1), from an imported state, after one
FP32 GPU round, and at the stopping round of a full decode."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.gf import hadamard  # noqa: E402
from oracle.sp import channel_prior, check_to_var, decode as odecode, run_rounds, tentative, var_to_check  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from tests._msg import TOL_FP32, fourier, from_state, to_state  # noqa: E402
from tests.test_gpu_parity import CASES, _dev, _setup  # noqa: E402

pytestmark = pytest.mark.gpu

PICK = [CASES[0], CASES[2], CASES[5], CASES[7], CASES[8]]


def _rel_err(got, ref, q=None):
    """max_x |got(x) - ref(x)| / max_x ref(x), per symbol: the worst, or its
    quantile q over symbols."""
    e = (np.abs(got - ref).max(-1) / ref.max(-1)).ravel()
    return float(e.max() if q is None else np.quantile(e, q))


def _metrics(got, ref):
    d = np.abs(got - ref)
    l1 = d.sum(-1)                                  # relative L1 error (pmfs sum to 1)
    rmax = d.max(-1) / ref.max(-1)
    big = ref >= 1e-2
    rent = (d[big] / ref[big]) if big.any() else np.zeros(1)
    return (f"L1 max {l1.max():.2e} p99.9 {np.quantile(l1, 0.999):.2e} | rel-to-max max {rmax.max():.2e} "
            f"p99.9 {np.quantile(rmax, 0.999):.2e} | entry rel (p>=1e-2) max {rent.max():.2e}")


@pytest.mark.parametrize("case", PICK, ids=lambda c: c[0])
def test_posterior_from_state_and_after_one_round(case):
    name, m, k, N, F, ebn0 = case
    print(f"[case] {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    ll = llr.astype(np.float64)
    p0 = channel_prior(ll, m)
    c2vs, _, _ = run_rounds(tc, ll, 3)
    # (1) posterior of the oracle's own state (rounded to FP32 words)
    for i in (0, 1, 2):
        got = D.posterior(gcode, L, _dev(to_state(c2vs[i]))).cpu().numpy()
        ref = tentative(tc, p0, c2vs[i]).post
        assert np.allclose(got.sum(-1), 1.0, atol=1e-12) and (got >= 0).all()
        err = _rel_err(got, ref)
        print(f"  state {i + 1}: posterior rel err {err:.2e}", flush=True)
        assert err < 1e-5
    # (2) one FP32 GPU round from the oracle's state (as FP32 words), then the
    # posterior.  Reference: the exact round from the same words, their pmfs
    # clamped at zero as the default variable node does (a rounded word vector
    # is not quite the transform of a nonnegative pmf).  Conditioning: the
    # kernel computes with P(z) = sign 2^-|w| and the channel pmf in FP32
    # (relative rounding), and forms each variable-to-check Fourier image
    # Y(z) / Y(0), |Y(z) / Y(0)| <= 1, in FP32, i.e. to an absolute 2^-24,
    # which for near-certain messages is a large relative error on 1 - |Y|.
    # The reference is recomputed with each P(z) and channel probability moved
    # by a random relative 2^-22 and each normalised Y(z) by a random
    # absolute 2^-22 (four units in the last place).  Every symbol whose
    # posterior moves by less than 1e-5 (relative to its largest probability)
    # is well-conditioned and held to 1e-4; the others (a small Y(0) where
    # prior and message disagree, or a posterior made of near-certain
    # messages' small probabilities) are counted and printed.
    H = hadamard(tc.q)
    rng = np.random.default_rng(5)

    def sign(shape):
        return np.where(rng.random(shape) < 0.5, -1.0, 1.0)

    def exact_post(P, prior, jiggle_v2c=False):
        p_in = np.maximum(P @ H, 0.0) / tc.q
        v2c = var_to_check(tc, prior, p_in)
        if jiggle_v2c:
            Y = fourier(v2c)
            Y = Y / Y[..., :1] + sign(Y.shape) * 2.0 ** -22
            Y[..., 0] = 1.0
            v2c = Y @ H / tc.q
        return tentative(tc, prior, check_to_var(tc, v2c)).post

    for i in (0, 1):
        words = to_state(c2vs[i])
        out = D.round_step(gcode, L, _dev(words), "fused")
        got = D.posterior(gcode, L, out["c2v"]).cpu().numpy()
        P = from_state(words)
        ref = exact_post(P, p0)
        moved = exact_post(P * (1 + sign(P.shape) * 2.0 ** -22), p0 * (1 + sign(p0.shape) * 2.0 ** -22), True)
        cond = np.abs(moved - ref).max(-1) / ref.max(-1)
        well = cond < 1e-5
        err = np.abs(got - ref).max(-1) / ref.max(-1)
        ill = err[~well]
        print(f"  GPU round {i + 2}: {_metrics(got, ref)}; well-conditioned {well.sum()}/{well.size} symbols, "
              f"max rel err on them {err[well].max():.2e}; ill-conditioned: max rel err {ill.max() if ill.size else 0:.2e}",
              flush=True)
        assert well.mean() > 0.9
        assert err[well].max() < TOL_FP32
        assert err.max() < 1e-2
    gcode.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("case", [CASES[0], CASES[5], CASES[7]], ids=lambda c: c[0])
def test_decode_posterior_at_stopping_round(case, prec):
    name, m, k, N, F, ebn0 = case
    print(f"[case] {name} {prec} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    dec = D.Decoder(gcode, F, prec, "fused")
    r = dec(L, 20)
    post = dec.posterior().cpu().numpy()
    iters = r["iters"].cpu().numpy()
    hard = r["hard"].cpu().numpy()
    assert np.allclose(post.sum(-1), 1.0, atol=1e-12) and (post >= 0).all()
    ref = odecode(tc, llr.astype(np.float64), 20)
    # frames the oracle decodes to a codeword and the GPU stops at the same
    # round with the same decision
    same = (iters == ref.iters) & (hard == ref.hard).all(1) & ref.converged
    # (16-bit storage may stop a round earlier or later)
    assert same.sum() >= (0.95 if prec == "fp32" else 0.75) * ref.converged.sum()
    sel = np.nonzero(same)[0]
    print(f"  {same.sum()} of {ref.converged.sum()} converged frames on the oracle's trajectory: "
          f"{_metrics(post[sel], ref.post[sel])}", flush=True)
    # the posterior's symbol decision is the oracle's
    assert np.array_equal(post[sel].argmax(-1), ref.post[sel].argmax(-1))
    # errors compound over the rounds of a decode.  16-bit storage rounds
    # every stored probability to a relative u (2^-11 FP16, 2^-8 BF16) each
    # round; the posterior multiplies two stored messages, so the median L1
    # distance is held to 4 u, the worst symbol to 40 u (FP32: 1e-4 and 1e-2)
    l1 = np.abs(post[sel] - ref.post[sel]).sum(-1)
    med, worst = {"fp32": (1e-4, 1e-2), "fp16": (4 * 2.0 ** -11, 40 * 2.0 ** -11),
                  "bf16": (4 * 2.0 ** -8, 40 * 2.0 ** -8)}[prec]
    assert np.median(l1) < med and l1.max() < worst
    gcode.close()


@pytest.mark.parametrize("case", [CASES[0], CASES[5], CASES[7]], ids=lambda c: c[0])
def test_symbol_map_and_soft_output(case):
    """Symbol-MAP decisions (argmax of the posterior, Sec. 3.1 Eq. (3)) and FP32
    soft output at the stopping round: the soft output is the FP64 posterior
    rounded, the decisions are the oracle's symbol-MAP decisions on the frames
    that follow its trajectory, away from near-ties."""
    name, m, k, N, F, ebn0 = case
    print(f"[case] symbols {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    dec = D.Decoder(gcode, F, "fp32", "fused")
    r = dec(L, 20)
    sym, soft = dec.symbols(soft=True)
    post64 = dec.posterior().cpu().numpy()
    sym, soft = sym.cpu().numpy(), soft.cpu().numpy()
    assert np.array_equal(soft, post64.astype(np.float32))
    assert np.array_equal(sym, post64.argmax(-1))
    ref = odecode(tc, llr.astype(np.float64), 20)
    same = (r["iters"].cpu().numpy() == ref.iters) & (r["hard"].cpu().numpy() == ref.hard).all(1)
    top2 = np.sort(ref.post, axis=-1)[..., -2:]
    clear = (top2[..., 1] - top2[..., 0]) > 1e-3          # symbols whose MAP is not a near-tie
    sel = same[:, None] & clear
    assert sel.sum() > 0.9 * same.sum() * N
    assert np.array_equal(sym[sel], ref.symmap[sel])
    gcode.close()


def test_posterior_after_batched_retirement_is_refused():
    """With BATCH_RETIRE a frame that stops inside a batched tail chunk has its
    messages overwritten by the chunk's later passes: the decode-time posterior
    of such a workspace is refused (E_UNSUPPORTED), a VALIDATION decode does not
    batch, and its posteriors equal those of a decode that never batched."""
    name, m, k, N, F, ebn0 = CASES[5]
    print(f"[case] batched posterior {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    gcode.set_tuning(tail_frames=1 << 20, tail_chunk=5)
    L = _dev(llr)
    dec = D.Decoder(gcode, F, "fp32", "fused")
    dec(L, 20)
    ref = dec.posterior().cpu().numpy()
    gcode.set_tuning(batch_retire=1)
    dec(L, 20)
    with pytest.raises(D.LdpcFdError) as ei:
        dec.posterior()
    assert ei.value.rc == D.E_UNSUPPORTED
    r = dec.decode_ex(L, 20, D.FLAG_VALIDATION)
    assert np.array_equal(r["posterior"].cpu().numpy(), ref)
    # a decode that does not batch makes the workspace readable again
    gcode.set_tuning(batch_retire=0)
    dec(L, 20)
    assert np.array_equal(dec.posterior().cpu().numpy(), ref)
    gcode.close()
