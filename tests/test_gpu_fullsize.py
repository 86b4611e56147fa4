"""Full-size cases in the launch configurations the benchmark times: the
GF(256) (2,8) N=512 precision configuration (8192 frames, FP32 / FP16 / BF16
storage) and the uneven three-code batch (11000 frames in one pool).  Outputs
are checked for properties that hold at any size (syndromes equal H x^, the
stopping rule), a frame sample against the FP64 oracle, and the pool against
the same codes decoded alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1008_4370_amd import autotune, serving, synth  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from tests._oracle_pool import oracle_decode_sample  # noqa: E402
from tests.test_gpu_parity import _check_outputs, _dev  # noqa: E402

pytestmark = pytest.mark.gpu


def test_gf256_n512_8192_frames_per_storage_type():
    """GF(256) (2,8) N=512 at 3.0 dB, 8192 frames: every storage type gives
    self-consistent outputs; on a 32-frame sample decoded by the FP64 oracle
    (spread over host processes: its direct q^2 convolutions take tens of
    seconds per GF(256) frame) frames that stop at the oracle's round carry its
    decision, and at least 30 (FP32, FP16) / 28 (BF16) of the 32 are identical
    to it; the FER of every storage type is printed beside the oracle
    sample's (the FER delta of this configuration against FP32 on all 8192
    frames; against the oracle only on the sample, whose few frames cannot
    resolve FERs near 1e-3)."""
    b = synth.make_batch("gf256_n512")
    F = b.llr.shape[0]
    print(f"[case] gf256_n512 {F} frames", flush=True)
    sample = np.linspace(0, F - 1, 32).astype(int)
    rhard, riters, rconv = oracle_decode_sample(b.code, b.llr[sample], 100)
    gcode = D.Code.from_synth(b.code)
    L = _dev(b.llr)
    fers = {}
    floor = {"fp32": 30, "fp16": 30, "bf16": 28}
    for prec in ("fp32", "fp16", "bf16"):
        autotune.apply(gcode, prec, F)
        r = {k: v.cpu().numpy() for k, v in D.decode(gcode, L, 100, prec=prec).items()}
        _check_outputs(r, b.enc, 100)
        fers[prec] = float(np.any(r["hard"] != b.cw, axis=1).mean())
        hard, iters = r["hard"][sample], r["iters"][sample]
        same_round = (iters == riters) & rconv
        ident = (iters == riters) & np.all(hard == rhard, axis=1)
        print(f"[gf256_n512] {prec}: FER {fers[prec]:.5f} (delta vs fp32 {fers[prec] - fers['fp32']:+.5f}); "
              f"oracle sample identical {ident.sum()}/32, sample FER GPU "
              f"{np.mean(np.any(hard != b.cw[sample], axis=1)):.3f} oracle {np.mean(~rconv):.3f}", flush=True)
        assert np.all(np.all(hard[same_round] == rhard[same_round], axis=1))
        assert ident.sum() >= floor[prec]
    gcode.close()
    assert fers["fp32"] < 0.01


def test_uneven_three_code_batch_in_one_pool_equals_each_code_alone():
    """3000 x GF(16) N=2048 + 6000 x GF(64) N=512 + 2000 x GF(256) k=16 N=256 at
    2.5 dB decoded together in one pool, as steps of 8 passes (the default:
    one graph replay per step runs every code, each code's kernel forms chosen
    from its active count), steps of 4 passes, one step of every pass (one
    graph launch) and staggered steps: per-frame results equal those of each
    code's batch decoded alone."""
    batches = [synth.make_batch(w) for w in ("gf16_n2048", "gf64_n512", "gf256_n256_k16")]
    print("[case] mixed batch 11000 frames", flush=True)
    codes = [D.Code.from_synth(b.code) for b in batches]
    for c, b in zip(codes, batches):
        autotune.apply(c, "fp32", b.llr.shape[0])
    llrs = [_dev(b.llr) for b in batches]
    pool = D.Pool(codes, [b.llr.shape[0] for b in batches], prec="fp32")
    runs = [serving.decode_mixed(pool, llrs, 100), serving.decode_mixed(pool, llrs, 100, 4),
            serving.decode_mixed(pool, llrs, 100, None)]
    pool.set_schedule(1, 4)
    runs.append(serving.decode_mixed(pool, llrs, 100))
    pool.set_schedule(1, 16)
    runs.append(serving.decode_mixed(pool, llrs, 100, None))
    pool.close()
    for i, (c, b, l) in enumerate(zip(codes, batches, llrs)):
        alone = {k: v.cpu().numpy() for k, v in D.decode(c, l, 100).items()}
        for mixed in runs:
            r = mixed[i]
            assert np.array_equal(r["hard"], alone["hard"])
            assert np.array_equal(r["iters"], alone["iters"])
            conv = (r["status"] & D.STATUS_CONVERGED) != 0
            assert np.array_equal(conv, (alone["status"] & D.STATUS_CONVERGED) != 0)
        print(f"[mixed] GF({b.code.q}) N={b.code.N}: FER {np.any(runs[0][i]['hard'] != b.cw, axis=1).mean():.4f}",
              flush=True)
    for c in codes:
        c.close()
