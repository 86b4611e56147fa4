"""ldpc_fd_round_noalloc (temporaries in the library's static device scratch,
no allocation inside the call) gives exactly what ldpc_fd_round gives, on two
calls in a row with the second smaller, and rejects rounds larger than its
scratch before enqueuing anything."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sp import TannerCode, run_rounds  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from paper_1008_4370_amd import synth  # noqa: E402
from tests._msg import to_state  # noqa: E402

pytestmark = pytest.mark.gpu


def _setup(m, k, N, F, seed):
    code = synth.make_code(N, k, m, seed_graph=700 + m, seed_labels=710 + k)
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, F, seed=seed)
    llr = synth.bpsk_awgn_llr(cw, m, 2.5, code.design_rate, seed=seed + 1)
    tc = TannerCode(code.M, code.N, code.m, code.row_ptr, code.col, code.val, code.poly)
    return code, llr, tc


@pytest.mark.parametrize("mode,prec", [("fused", "fp32"), ("fused", "fp16"), ("fused", "bf16"), ("plain", "fp32"),
                                       ("logsp", "fp32")])
def test_noalloc_round_equals_round(mode, prec):
    m, k, N = 6, 6, 60
    code, llr, tc = _setup(m, k, N, 37, seed=11)
    print(f"[case] noalloc {mode} {prec} GF(64) N=60", flush=True)
    gcode = D.Code.from_synth(code)
    L = torch.from_numpy(llr).cuda()
    c2vs, _, _ = run_rounds(tc, llr.astype(np.float64), 2)
    if mode == "logsp":
        state = np.log2(np.maximum(c2vs[0] / c2vs[0].max(-1, keepdims=True), 2.0 ** -200)).astype(np.float32)
    else:
        state = to_state(c2vs[0])
    S = torch.from_numpy(state).cuda()
    for F in (37, 20):   # second call smaller: the scratch keeps the first call's contents
        for st in (None, S[:F]):
            ref = D.round_step(gcode, L[:F], st, mode, prec)
            got = D.round_step_noalloc(gcode, L[:F], st, mode, prec)
            torch.cuda.synchronize()
            for key in ("c2v", "v2c", "hard", "fsynd", "synd"):
                if ref[key] is None:
                    assert got[key] is None
                    continue
                assert torch.equal(got[key], ref[key]), (F, st is None, key)
    gcode.close()


def test_noalloc_round_rejects_more_than_its_scratch():
    m, k, N = 6, 6, 60
    code, llr, tc = _setup(m, k, N, 4, seed=13)
    gcode = D.Code.from_synth(code)
    E, q = gcode.E, gcode.q
    # 16-bit storage stages the imported and exported state: 2 * 2 * E * q bytes
    # per frame, so 64 MiB holds fewer than 2200 GF(64) N=60 frames
    F = 2500
    L = torch.zeros((F, N, m), dtype=torch.float32, device="cuda")
    out = torch.empty((F, E, q), dtype=torch.float32, device="cuda")
    marker = out.clone().fill_(3.0)
    out.copy_(marker)
    with pytest.raises(D.LdpcFdError) as ei:
        D._check(D.lib().ldpc_fd_round_noalloc(gcode.handle, F, D._ptr(L), None, None, D._ptr(out), None, None,
                                               None, D.MODE["fused"], D.PREC["fp16"], D._stream()))
    assert ei.value.rc == D.E_NOMEM and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.equal(out, marker)   # nothing was enqueued
    # the same round at FP32 storage fits and runs
    r = D.round_step_noalloc(gcode, L[:1000], None, "fused", "fp32")
    torch.cuda.synchronize()
    assert bool(torch.isfinite(r["c2v"]).all())
    gcode.close()
