"""GPU parity: the HIP decoder (through the C-ABI) against the FP64 oracle on the
same seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.gf import hadamard  # noqa: E402
from oracle.sp import (TannerCode, channel_prior, check_to_var, decode as odecode, run_rounds,  # noqa: E402
                       tentative, var_to_check)
from paper_1008_4370_amd import decoder as D  # noqa: E402
from paper_1008_4370_amd import synth  # noqa: E402
from tests._oracle_pool import oracle_decode_sample  # noqa: E402
from tests._msg import (TOL_FP32, fourier, from_state, fsynd_near_tie, near_tie_bits,  # noqa: E402
                        store_pmf, to_state)

pytestmark = pytest.mark.gpu

# (name, m, k, N, frames, EbN0): frame counts leave a ragged last group for every
# lane geometry; rows of weight <= 8 and 9..16 exercise both kernel families.
CASES = [
    ("gf4_k4_n96", 2, 4, 96, 70, 2.0),
    ("gf8_k6_n30", 3, 6, 30, 67, 2.5),
    ("gf16_k4_n64", 4, 4, 64, 69, 2.0),
    ("gf16_k12_n48", 4, 12, 48, 21, 3.5),
    ("gf32_k5_n40", 5, 5, 40, 35, 2.5),
    ("gf64_k6_n60", 6, 6, 60, 37, 2.5),
    ("gf128_k4_n24", 7, 4, 24, 19, 2.0),
    ("gf256_k8_n24", 8, 8, 24, 9, 3.0),
    ("gf256_k16_n32", 8, 16, 32, 5, 3.0),
]


def _setup(m, k, N, F, ebn0, seed=0):
    code = synth.make_code(N, k, m, seed_graph=900 + m + seed, seed_labels=950 + k + seed)
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, F, seed=5 + seed)
    llr = synth.bpsk_awgn_llr(cw, m, ebn0, code.design_rate, seed=6 + seed)
    tc = TannerCode(code.M, code.N, code.m, code.row_ptr, code.col, code.val, code.poly)
    return code, enc, cw, llr, tc


def _dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("mode", ["plain", "fused", "fused+precise", "fused+butterfly"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_one_round_message_parity(case, mode):
    """From the same imported state, one GPU round matches the oracle's round:
    messages within 1e-4 in the linear Fourier domain, decisions equal except
    near-ties, direct syndromes bit-exact for the GPU's own decisions."""
    name, m, k, N, F, ebn0 = case
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    print(f"[case] {name} mode={mode} F={F}", flush=True)
    gcode = D.Code.from_synth(code)
    if mode in ("fused+precise", "fused+butterfly"):
        gcode.set_tuning(precise=1 if mode == "fused+precise" else 0)
        mode = "fused"
    L = _dev(llr)
    c2vs, v2cs, decs = run_rounds(tc, llr.astype(np.float64), 3)
    # round 0 -> 1 (initial messages)
    out = D.round_step(gcode, L, None, mode)
    torch.cuda.synchronize()
    assert np.abs(from_state(out["c2v"].cpu().numpy()) - fourier(c2vs[0])).max() < TOL_FP32
    if mode == "plain":
        p0 = channel_prior(llr.astype(np.float64), m)[:, tc.edge_var]
        assert np.abs(from_state(out["v2c"].cpu().numpy()) - fourier(p0)).max() < TOL_FP32
    for i in (0, 1):
        out = D.round_step(gcode, L, _dev(to_state(c2vs[i])), mode)
        torch.cuda.synchronize()
        err_c = np.abs(from_state(out["c2v"].cpu().numpy()) - fourier(c2vs[i + 1])).max()
        assert err_c < TOL_FP32, err_c
        if mode == "plain":
            err_v = np.abs(from_state(out["v2c"].cpu().numpy()) - fourier(v2cs[i])).max()
            assert err_v < TOL_FP32, err_v
        hard = out["hard"].cpu().numpy()
        d = decs[i]
        ok = near_tie_bits(d.qbits)
        assert np.array_equal(hard[~ok], d.hard[~ok])
        assert np.array_equal(out["synd"].cpu().numpy().astype(np.int64), enc.syndrome(hard.astype(np.int64)))
        fs_ok = fsynd_near_tie(tc, d.post)
        fs = out["fsynd"].cpu().numpy()
        assert np.array_equal(fs[~fs_ok], d.fsynd[~fs_ok])
    gcode.close()


# 16-bit storage holds each check-to-variable message as q times its pmf
# (the inverse transform of P, clamped at zero) rounded to FP16 or BF16, and
# the FUSED pass reads it with the default variable node (PRECISE = 2), the
# form bench.py, fer.py and the serving loop run.  Parity: one GPU round from
# an imported state against the FP64 oracle applied to the state as stored
# (the same clamped, rounded pmfs), its output rounded the same way.  Both
# sides then take identical, nonnegative input pmfs, so the arithmetic part of
# the difference is the FP32 one (TOL_FP32); the rounding of the output can
# differ by one unit in the last place of an entry where the FP32 and FP64
# values straddle a rounding boundary, which moves the normalised Fourier
# image by at most u * sum_x p(x) = u (u = 2^-11 FP16, 2^-8 BF16).  The bound
# holds on every entry (no percentile).
STORAGE_U = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[5], CASES[6], CASES[7], CASES[8]], ids=lambda c: c[0])
def test_one_round_storage_parity(case, prec):
    name, m, k, N, F, ebn0 = case
    print(f"[case] storage {name} {prec} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    assert gcode.get_tuning()["precise"] == 2
    L = _dev(llr)
    ll = llr.astype(np.float64)
    c2vs, _, _ = run_rounds(tc, ll, 3)
    p0 = channel_prior(ll, m)
    H = hadamard(tc.q)
    errs, errs_store = [], []
    for i in (0, 1):
        w = to_state(c2vs[i])
        out = D.round_step(gcode, L, _dev(w), "fused", prec)
        torch.cuda.synchronize()
        got = from_state(out["c2v"].cpu().numpy())
        # the oracle on the state as stored, its output rounded as stored
        p_in = store_pmf(from_state(w) @ H.T, prec) / tc.q
        nxt = check_to_var(tc, var_to_check(tc, p0, p_in))
        want = fourier(store_pmf(tc.q * nxt, prec))
        want = want / want[..., :1]
        err = np.abs(got - want).max()
        errs.append(err)
        errs_store.append(np.abs(got - fourier(c2vs[i + 1])).max())
        assert err < TOL_FP32 + STORAGE_U[prec], (i, err)
        # the decision of the imported round: the oracle's on the stored state,
        # except bits near a tie; direct syndromes bit-exact
        d = tentative(tc, p0, p_in)
        hard = out["hard"].cpu().numpy()
        ok = near_tie_bits(d.qbits)
        assert np.array_equal(hard[~ok], d.hard[~ok])
        assert np.array_equal(out["synd"].cpu().numpy().astype(np.int64), enc.syndrome(hard.astype(np.int64)))
    print(f"[storage] {name} {prec}: vs stored-state oracle max {max(errs):.3e} "
          f"(bound {TOL_FP32 + STORAGE_U[prec]:.2e}); storage error vs FP64 oracle {max(errs_store):.3e}",
          flush=True)
    gcode.close()


def _full_run(code, llr, max_iter, prec, mode):
    gcode = D.Code.from_synth(code)
    r = D.decode(gcode, _dev(llr), max_iter, prec=prec, mode=mode)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items()}
    gcode.close()
    return out


def _check_outputs(out, enc, max_iter):
    hard = out["hard"].astype(np.int64)
    assert np.array_equal(out["synd"].astype(np.int64), enc.syndrome(hard))
    conv = (out["status"] & D.STATUS_CONVERGED) != 0
    assert np.all(out["synd"][conv] == 0)
    assert np.all((out["iters"] >= 1) & (out["iters"] <= max_iter))
    assert np.all(out["iters"][~conv] == max_iter)
    return conv


@pytest.mark.parametrize("mode", ["plain", "fused"])
def test_full_run_parity_gf4_n96_1000_frames(mode):
    """GF(4) (2,4) N=96, 1000 frames at 2.0 dB, max 50 rounds: per-frame results
    match the oracle; trajectories that meet a near-tie may diverge (allowed for
    at most 1% of frames)."""
    b = synth.make_batch("gf4_n96")
    tc = TannerCode(b.code.M, b.code.N, b.code.m, b.code.row_ptr, b.code.col, b.code.val, b.code.poly)
    print(f"[case] gf4_n96 full mode={mode}", flush=True)
    ref = odecode(tc, b.llr, 50)
    out = _full_run(b.code, b.llr, 50, "fp32", mode)
    conv = _check_outputs(out, b.enc, 50)
    same = (np.all(out["hard"] == ref.hard, axis=1) & (out["iters"] == ref.iters) & (conv == ref.converged))
    assert same.mean() >= 0.99, same.mean()
    mism = (out["status"] & D.STATUS_MISMATCH) != 0
    assert (mism == ref.mismatch)[same].mean() >= 0.99


def test_plain_and_fused_agree_and_are_deterministic():
    b = synth.make_batch("gf4_n96", frames=300)
    a = _full_run(b.code, b.llr, 30, "fp32", "fused")
    a2 = _full_run(b.code, b.llr, 30, "fp32", "fused")
    p = _full_run(b.code, b.llr, 30, "fp32", "plain")
    for k in a:
        assert np.array_equal(a[k], a2[k]), k
    same = np.all(a["hard"] == p["hard"], axis=1) & (a["iters"] == p["iters"])
    assert same.mean() >= 0.99


def test_codeword_shift_symmetry_on_gpu():
    b = synth.make_batch("gf4_n96", frames=200)
    c = synth.random_codewords(b.enc, 1, seed=77)[0]
    flip = (1 - 2 * ((c[None, :, None] >> np.arange(b.code.m)) & 1)).astype(np.float32)
    for mode in ("plain", "fused"):
        r1 = _full_run(b.code, b.llr, 30, "fp32", mode)
        r2 = _full_run(b.code, b.llr * flip, 30, "fp32", mode)
        assert np.array_equal(r1["iters"], r2["iters"])
        assert np.array_equal(r1["hard"] ^ c[None, :].astype(np.uint8), r2["hard"])


# 32 frames evenly spaced over the 4096-frame batch, decoded once by the
# oracle (spread over host processes) for every storage type's test.
FULL_SAMPLE = np.linspace(0, 4095, 32).astype(int)
# fraction of the sample whose hard decisions and stopping round equal the
# oracle's, per storage type (FP32: every frame)
FULL_AGREE = {"fp32": 1.0, "fp16": 0.9, "bf16": 0.8}


@pytest.fixture(scope="module")
def gf64_n1000_oracle():
    b = synth.make_batch("gf64_n1000", point=2)
    print("[oracle] GF(64) N=1000, 32 sampled frames", flush=True)
    return b, oracle_decode_sample(b.code, b.llr[FULL_SAMPLE], 100)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_gf64_n1000_full_size_sampled_parity(prec, gf64_n1000_oracle):
    """GF(64) (2,6) N=1000 at 2.5 dB with 4096 frames in the fused launch the
    benchmark times: every frame's outputs are self-consistent (syndromes are
    H x^ exactly, stop rule holds); on a 32-frame sample decoded by the FP64
    oracle, every frame that stops at the oracle's round with a passed
    codeword test carries the oracle's decision, and the fraction of sampled
    frames identical to the oracle (decision and round) is at least
    FULL_AGREE[prec]."""
    b, (rhard, riters, rconv) = gf64_n1000_oracle
    print(f"[case] gf64_n1000 full prec={prec}", flush=True)
    out = _full_run(b.code, b.llr, 100, prec, "fused")
    conv = _check_outputs(out, b.enc, 100)
    fer = np.any(out["hard"] != b.cw, axis=1).mean()
    hard, iters = out["hard"][FULL_SAMPLE], out["iters"][FULL_SAMPLE]
    same_round = (iters == riters) & rconv
    ident = (iters == riters) & np.all(hard == rhard, axis=1)
    print(f"[full-size] gf64_n1000 {prec}: converged {conv.mean():.4f} FER {fer:.4f} "
          f"mean iters {out['iters'].mean():.2f}; oracle sample identical {ident.mean():.3f} "
          f"(same round {np.mean(iters == riters):.3f}; oracle sample FER {np.mean(~rconv):.3f})", flush=True)
    assert conv.mean() > 0.9
    assert np.all(np.all(hard[same_round] == rhard[same_round], axis=1))
    assert ident.mean() >= FULL_AGREE[prec]


def test_edge_cases():
    b = synth.make_batch("gf4_n96", frames=5)
    gcode = D.Code.from_synth(b.code)
    # zero frames is a no-op
    dec = D.Decoder(gcode, 5, "fp32", "fused")
    empty = torch.empty((0, b.code.N, b.code.m), dtype=torch.float32, device="cuda")
    rc = D.lib().ldpc_fd_decode(gcode.handle, 0, D._ptr(empty), 10, 0, 1, None, None, None, None, None, 0, None)
    assert rc == D.OK
    # all-zero LLRs: uniform posteriors, zero word, stops at round 1
    z = torch.zeros((5, b.code.N, b.code.m), dtype=torch.float32, device="cuda")
    for mode in ("plain", "fused"):
        r = D.decode(gcode, z, 10, mode=mode)
        assert int(r["hard"].max()) == 0 and bool((r["iters"] == 1).all())
    # max_iter = 1
    r = D.decode(gcode, _dev(b.llr), 1)
    assert bool((r["iters"] == 1).all())
    # workspace too small / bad precision
    rc = D.lib().ldpc_fd_decode(gcode.handle, 5, D._ptr(z), 10, 0, 1, D._ptr(dec.hard), D._ptr(dec.synd),
                                D._ptr(dec.iters), D._ptr(dec.status), D._ptr(dec.workspace), 16, None)
    assert rc == D.E_NOMEM
    rc = D.lib().ldpc_fd_decode(gcode.handle, 5, D._ptr(z), 10, 7, 1, D._ptr(dec.hard), D._ptr(dec.synd),
                                D._ptr(dec.iters), D._ptr(dec.status), D._ptr(dec.workspace), dec.ws_bytes, None)
    assert rc == D.E_INVALID
    gcode.close()


def test_graph_replay_matches_eager_launches():
    """Captured round chunks replayed several times, with eager decodes and
    synchronisations in between, give exactly the eager results every time."""
    b = synth.make_batch("gf64_n1000", point=1, frames=300)
    gcode = D.Code.from_synth(b.code)
    L = _dev(b.llr)
    gcode.set_tuning(graphs=0)
    ref = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 40, prec="fp32").items()}
    gcode.set_tuning(graphs=1)
    dec = D.Decoder(gcode, 300, "fp32", "fused")
    for rep in range(4):
        out = {k: v.cpu().numpy() for k, v in dec(L, 40).items()}
        for k in ref:
            assert np.array_equal(out[k], ref[k]), (rep, k)
        gcode.set_tuning(graphs=0)
        eager = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 40, prec="fp32").items()}
        assert all(np.array_equal(eager[k], ref[k]) for k in ref)
        gcode.set_tuning(graphs=1)
    # longer captured chunks for the tail passes (tuning key TAIL_CHUNK): the
    # same results, passes after the last frame stops doing nothing
    for tc in (1, 5, 32):
        gcode.set_tuning(tail_chunk=tc, tail_frames=64)
        out = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 40, prec="fp32").items()}
        for k in ref:
            assert np.array_equal(out[k], ref[k]), (tc, k)
    # a first chunk of its own length (tuning key FIRST_CHUNK) with short later
    # chunks and a tail threshold above 128, so that tail chunks start with
    # more than 128, at most 128 and at most 32 active frames (the
    # edge-parallel grid sized by that count), with and without batched
    # retirement, replayed and launched eagerly
    for fc, ch, br, g in ((3, 1, 0, 1), (6, 2, 1, 1), (5, 2, 1, 0), (9, 3, 1, 1)):
        gcode.set_tuning(first_chunk=fc, chunk=ch, tail_frames=200, tail_chunk=0, batch_retire=br, graphs=g)
        out = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 40, prec="fp32").items()}
        for k in ref:
            assert np.array_equal(out[k], ref[k]), (fc, ch, br, g, k)
    gcode.close()


def test_precise_variable_node_when_channel_and_messages_disagree():
    """The variable node where reliable channel bits contradict near-certain
    check messages: the prior convolution cancels the leading 1s, and the result
    is made of the small differences from certainty.  Messages are
    near-deterministic pmfs (1 - eps on a random symbol, eps in 1e-6..1e-3
    spread over the others) and channel bits have |L| in 8..16.  With the FP64
    variable node (tuning key PRECISE) one GPU round matches the oracle to 1e-4
    on the well-conditioned entries; the FP32 form's error is printed."""
    m, k, N, F = 6, 6, 60, 8
    code, enc, cw, llr, tc = _setup(m, k, N, F, 2.5)
    q = tc.q
    print(f"[case] conflict gf64_k6_n60 F={F}", flush=True)
    rng = np.random.default_rng(123)
    eps = 10.0 ** rng.uniform(-6, -3, size=(F, tc.E, 1))
    tail = rng.random((F, tc.E, q))
    star = rng.integers(0, q, size=(F, tc.E))
    tail[np.arange(F)[:, None], np.arange(tc.E)[None, :], star] = 0.0
    pmf = eps * tail / tail.sum(-1, keepdims=True)
    pmf[np.arange(F)[:, None], np.arange(tc.E)[None, :], star] = 1.0 - eps[..., 0]
    llr2 = (rng.uniform(8.0, 16.0, size=(F, N, m)) * rng.choice([-1.0, 1.0], size=(F, N, m))).astype(np.float32)
    p0 = channel_prior(llr2.astype(np.float64), m)
    words = to_state(pmf)
    H = hadamard(tc.q)

    def oracle_round(w):
        return fourier(check_to_var(tc, var_to_check(tc, p0, from_state(w) @ H / tc.q)))

    # The oracle takes the state the GPU gets (the FP32 words).  Entries whose
    # exact value moves by more than 1e-6 when every word magnitude moves by one
    # ulp are ill-conditioned for any arithmetic and are left out (~2% here).
    ref = oracle_round(words)
    mag = np.abs(words)
    toward = np.where(rng.random(words.shape) < 0.5, np.inf, 0.0).astype(np.float32)
    bumped = np.copysign(np.where(mag == 0, mag, np.nextafter(mag, toward)), words).astype(np.float32)
    well = np.abs(oracle_round(bumped) - ref) < 1e-6
    gcode = D.Code.from_synth(code)
    errs = {}
    for precise in (0, 1, 2):
        gcode.set_tuning(precise=precise)
        out = D.round_step(gcode, _dev(llr2), _dev(words), "fused")
        torch.cuda.synchronize()
        errs[precise] = float(np.abs(from_state(out["c2v"].cpu().numpy()) - ref)[well].max())
    print(f"  {well.mean():.1%} of entries well-conditioned; one-round max |dP| on them: "
          f"FP32 variable node {errs[0]:.2e}, FP64 variable node {errs[1]:.2e}, "
          f"FP32 probability-domain prior {errs[2]:.2e}", flush=True)
    assert well.mean() > 0.9
    assert errs[1] < TOL_FP32
    assert errs[1] <= errs[0]
    gcode.close()


MFMA_CASES = [CASES[2], CASES[4], CASES[5]]   # q = 16, 32, 64 with 4 lanes per frame


@pytest.mark.parametrize("case", MFMA_CASES, ids=lambda c: c[0])
def test_decision_on_matrix_cores(case):
    """Decision transforms as FP16 MFMAs (tuning key DECISION_MFMA): the messages
    are bit-identical to the VALU decision's round (the decision does not feed
    them); hard decisions equal the oracle's except bits whose posterior value
    is within FP16 reach of a tie (|q| < 1e-2), and at most 1% of symbols differ."""
    name, m, k, N, F, ebn0 = case
    print(f"[case] mfma decision {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    gcode.set_tuning(lane_entries=(1 << m) // 4, precise=0)   # MFMA decision: butterfly form
    L = _dev(llr)
    c2vs, _, decs = run_rounds(tc, llr.astype(np.float64), 3)
    for i in (0, 1):
        st = _dev(to_state(c2vs[i]))
        gcode.set_tuning(decision_mfma=0)
        base = D.round_step(gcode, L, st, "fused")
        gcode.set_tuning(decision_mfma=1)
        out = D.round_step(gcode, L, st, "fused")
        torch.cuda.synchronize()
        assert torch.equal(out["c2v"], base["c2v"])
        hard = out["hard"].cpu().numpy()
        d = decs[i]
        tie = (np.abs(d.qbits) < 1e-2).any(-1)
        assert np.array_equal(hard[~tie], d.hard[~tie])
        assert (hard == d.hard).mean() >= 0.99
        assert np.array_equal(out["synd"].cpu().numpy().astype(np.int64), enc.syndrome(hard.astype(np.int64)))
    gcode.close()


def test_decision_on_matrix_cores_full_decode():
    """Full decodes with the MFMA decision stop at the same round with the same
    output as the VALU decision for >= 98% of frames (GF(64) N=60, 2.5 dB)."""
    name, m, k, N, F, ebn0 = CASES[5]
    code, enc, cw, llr, tc = _setup(m, k, N, 256, ebn0)
    gcode = D.Code.from_synth(code)
    gcode.set_tuning(lane_entries=16, precise=0)   # MFMA decision: butterfly form
    L = _dev(llr)
    res = []
    for mf in (0, 1):
        gcode.set_tuning(decision_mfma=mf)
        r = D.decode(gcode, L, 50, prec="fp32", mode="fused")
        res.append({k2: v.cpu().numpy() for k2, v in r.items()})
    same = (res[0]["iters"] == res[1]["iters"]) & (res[0]["hard"] == res[1]["hard"]).all(1)
    print(f"  identical frames {same.mean():.3f}", flush=True)
    assert same.mean() >= 0.98
    gcode.close()


@pytest.mark.parametrize("case", [CASES[1], CASES[3], CASES[5], CASES[8]], ids=lambda c: c[0])
@pytest.mark.parametrize("precise", [0, 1, 2])
def test_edge_parallel_tail_pass_is_identical(case, precise):
    """Chunks with few active frames run the edge-parallel pass (one wavefront
    per edge); it sums a check's magnitudes in the same order as the
    check-serial pass, so decodes are bit-identical with it on and off (forced
    here for every chunk by a large tail threshold), and with no tail form at
    all (threshold 0: the full-batch pass and the two-launch syndromes and
    retirement throughout, where the tail runs them as one launch once at most
    128 frames are active)."""
    name, m, k, N, F, ebn0 = case
    print(f"[case] split tail {name} precise={precise} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    gcode.set_tuning(tail_frames=1 << 20, tail_entries=4, precise=precise, chunk=3)
    L = _dev(llr)
    # 16-bit storage is built for the default variable node only
    precs = ("fp32", "fp16", "bf16") if precise == 2 else ("fp32",)
    res = {}
    for split, batch in ((0, 1), (1, 0), (1, 1)):
        gcode.set_tuning(tail_split=split, batch_retire=batch)
        for prec in precs:
            r = D.decode(gcode, L, 30, prec=prec, mode="fused")
            res[(split, batch), prec] = {k2: v.cpu().numpy() for k2, v in r.items()}
    gcode.set_tuning(tail_frames=0)
    for prec in precs:
        r = D.decode(gcode, L, 30, prec=prec, mode="fused")
        res["none", prec] = {k2: v.cpu().numpy() for k2, v in r.items()}
    for prec in precs:
        for key in ("hard", "synd", "iters", "status"):
            assert np.array_equal(res[(0, 1), prec][key], res[(1, 0), prec][key]), (prec, key)
            assert np.array_equal(res[(1, 0), prec][key], res[(1, 1), prec][key]), (prec, key, "batched")
            assert np.array_equal(res["none", prec][key], res[(1, 1), prec][key]), (prec, key, "no tail")
    gcode.close()


@pytest.mark.parametrize("case", [CASES[5], CASES[8]], ids=lambda c: c[0])
def test_batched_retirement_from_mid_decode(case):
    """A batch larger than 128 frames retires after every pass until at most
    128 frames are active, then keeps each tail chunk's decisions and retires
    once per chunk (every frame still stops at its first codeword round):
    decodes identical to retiring after every pass, for chunks shorter than,
    equal to and unrelated to the frames' stopping rounds, with and without
    early stopping."""
    name, m, k, N, F, ebn0 = case
    F = 300
    print(f"[case] batched retirement {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0 - 0.5, seed=3)
    gcode = D.Code.from_synth(code)
    gcode.set_tuning(tail_frames=1 << 20, tail_entries=4, chunk=2)
    L = _dev(llr)
    gcode.set_tuning(batch_retire=0)
    ref = {k2: v.cpu().numpy() for k2, v in D.decode(gcode, L, 40, prec="fp32", mode="fused").items()}
    _check_outputs(ref, enc, 40)
    assert len(np.unique(ref["iters"])) > 3
    gcode.set_tuning(batch_retire=1)
    for tch in (1, 3, 7, 32):
        gcode.set_tuning(tail_chunk=tch)
        out = {k2: v.cpu().numpy() for k2, v in D.decode(gcode, L, 40, prec="fp32", mode="fused").items()}
        for key in ("hard", "synd", "iters", "status"):
            assert np.array_equal(ref[key], out[key]), (tch, key)
    dec = D.Decoder(gcode, F, "fp32", "fused")
    for batch in (0, 1):
        gcode.set_tuning(batch_retire=batch, tail_chunk=7)
        r = dec.decode_ex(L[:100].contiguous(), 40, D.FLAG_NO_EARLY_STOP)   # at most 128 frames: batched
        res = {k2: v.cpu().numpy() for k2, v in r.items()}
        if batch == 0:
            ref_ne = res
        else:
            for key in ("hard", "synd", "iters", "status"):
                assert np.array_equal(ref_ne[key], res[key]), ("no early stop", key)
    assert np.all(ref_ne["iters"] == 40)
    gcode.close()


def _qsc_prior(cw, q, eps, seed):
    """q-ary symmetric channel: the received symbol is the sent one with
    probability 1 - eps, else uniform over the others; prior of each symbol."""
    rng = np.random.default_rng(seed)
    F, N = cw.shape
    flip = rng.random((F, N)) < eps
    other = (cw + rng.integers(1, q, size=(F, N))) % q
    rx = np.where(flip, other, cw)
    p0 = np.full((F, N, q), eps / (q - 1), dtype=np.float32)
    np.put_along_axis(p0, rx[..., None], np.float32(1.0 - eps), axis=2)
    return p0


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[5], CASES[8]], ids=lambda c: c[0])
def test_symbol_prior_decoding(case):
    """Decoding from symbol priors (ldpc_fd_decode_prior): with the BPSK prior it
    follows the LLR decode (>= 95% of frames identical), and on a q-ary
    symmetric channel it matches the oracle run on the same priors."""
    name, m, k, N, F, ebn0 = case
    print(f"[case] symbol prior {name} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    dec = D.Decoder(gcode, F, "fp32", "fused")
    a = {k2: v.cpu().numpy().copy() for k2, v in dec(_dev(llr), 30).items()}
    p0 = channel_prior(llr.astype(np.float64), m).astype(np.float32)
    b = {k2: v.cpu().numpy().copy() for k2, v in dec.decode_prior(_dev(p0), 30).items()}
    same = (a["iters"] == b["iters"]) & (a["hard"] == b["hard"]).all(1)
    assert same.mean() >= 0.95   # FP32 trajectories of the two arithmetic routes may part
    assert np.array_equal(b["synd"].astype(np.int64), enc.syndrome(b["hard"].astype(np.int64)))
    eps = 0.08
    pq = _qsc_prior(cw, tc.q, eps, seed=17)
    g = {k2: v.cpu().numpy().copy() for k2, v in dec.decode_prior(_dev(pq), 30).items()}
    ref = odecode(tc, None, 30, prior=pq.astype(np.float64))
    same = (g["iters"] == ref.iters) & (g["hard"] == ref.hard).all(1)
    print(f"  BPSK prior vs LLR identical {np.mean((a['iters'] == b['iters']) & (a['hard'] == b['hard']).all(1)):.3f};"
          f" q-SC vs oracle identical {same.mean():.3f}, oracle FER {np.mean((ref.hard != cw).any(1)):.3f}", flush=True)
    assert same.mean() >= 0.95
    gcode.close()


def test_unbuilt_combinations_are_rejected():
    """16-bit storage holds message pmfs, which only the default variable node
    reads: the butterfly and FP64 forms with FP16/BF16 storage, and symbol
    priors with 16-bit storage, are not built and the entry points return
    E_UNSUPPORTED (every form takes FP32 storage)."""
    code, enc, cw, llr, tc = _setup(6, 6, 60, 4, 2.5)
    gcode = D.Code.from_synth(code)
    for precise in (0, 1):
        gcode.set_tuning(precise=precise)
        for prec in ("fp16", "bf16"):
            with pytest.raises(D.LdpcFdError) as ei:
                D.decode(gcode, _dev(llr), 10, prec=prec, mode="fused")
            assert ei.value.rc == -2
            with pytest.raises(D.LdpcFdError) as ei:
                D.round_step(gcode, _dev(llr), None, "fused", prec)
            assert ei.value.rc == -2
            with pytest.raises(D.LdpcFdError) as ei:
                D.Pool([gcode], [4], prec)
            assert ei.value.rc == -2
    gcode.set_tuning(precise=2)
    dec = D.Decoder(gcode, 4, "fp16", "fused")
    p0 = channel_prior(llr.astype(np.float64), 6).astype(np.float32)
    with pytest.raises(D.LdpcFdError) as ei:
        dec.decode_prior(_dev(p0), 10)
    assert ei.value.rc == -2
    gcode.close()


def test_probability_domain_prior_decodes_like_the_oracle():
    """GF(64) (2,6) N=1000, 4096 frames at 2.5 dB: the FP32 variable node through
    the convolution theorem with a clamped message pmf (PRECISE = 2, the
    default) fails on fewer than half as many frames as the FP32 butterfly form
    (PRECISE = 0), its outputs are
    self-consistent, and the frames the butterfly form fails are decoded as the
    FP64 oracle decodes them on most (>= 70%) of those frames (the oracle
    itself decodes all but one of them)."""
    b = synth.make_batch("gf64_n1000", point=2)
    print("[case] gf64_n1000 full precise=2", flush=True)
    gcode = D.Code.from_synth(b.code)
    L = _dev(b.llr)
    gcode.set_tuning(precise=0)
    base = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 100).items()}
    gcode.set_tuning(precise=2)
    out = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 100).items()}
    gcode.close()
    _check_outputs(out, b.enc, 100)
    fer0 = np.any(base["hard"] != b.cw, axis=1).mean()
    fer2 = np.any(out["hard"] != b.cw, axis=1).mean()
    print(f"[prob prior] FER butterfly form {fer0:.5f} -> {fer2:.5f}", flush=True)
    assert fer2 < 0.5 * fer0
    bad = np.nonzero(np.any(base["hard"] != b.cw, axis=1))[0][:16]
    tc = TannerCode(b.code.M, b.code.N, b.code.m, b.code.row_ptr, b.code.col, b.code.val, b.code.poly)
    ref = odecode(tc, b.llr[bad], 100)
    agree = np.all(out["hard"][bad] == ref.hard, axis=1)
    print(f"[prob prior] on {len(bad)} frames the butterfly form fails: equal to the oracle {agree.mean():.3f}",
          flush=True)
    assert agree.mean() >= 0.7


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("case", [CASES[2], CASES[5], CASES[6], CASES[8]], ids=lambda c: c[0])
def test_lane_geometries_give_identical_results(case, prec):
    """Every kernel variant (4, 8 or 16 entries of a message per lane, and the
    few-frames variant the decoder switches to mid-decode) forms the same FP32
    values in the same order, so decodes are bit-identical whatever the
    variant (the autotuner only changes speed)."""
    name, m, k, N, F, ebn0 = case
    print(f"[case] lane geometries {name} {prec} F={F}", flush=True)
    code, enc, cw, llr, tc = _setup(m, k, N, F, ebn0)
    gcode = D.Code.from_synth(code)
    L = _dev(llr)
    choices = [e for e in (4, 8, 16) if e <= tc.q and not (e == 16 and (m == 8 or k > 8))]
    res = []
    for e in choices:
        gcode.set_tuning(lane_entries=e, tail_frames=0)
        res.append({k2: v.cpu().numpy() for k2, v in D.decode(gcode, L, 30, prec=prec).items()})
    for r in res[1:]:
        for key in ("hard", "synd", "iters", "status"):
            assert np.array_equal(res[0][key], r[key]), key
    gcode.close()
