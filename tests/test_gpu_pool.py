"""Decoding pool (continuous batching over several codes): every frame's result
is identical whether it is decoded alone (ldpc_fd_decode) or in a mix of codes
admitted at staggered times; slot accounting; results against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.sp import TannerCode, decode as odecode  # noqa: E402
from paper_1008_4370_amd import decoder as D  # noqa: E402
from paper_1008_4370_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

# small members of the three code families of the mixed workload
MIX = [("gf16_k4", 4, 4, 128, 2.0), ("gf64_k6", 6, 6, 60, 2.5), ("gf256_k16", 8, 16, 32, 3.0)]


def _family(m, k, N, ebn0, F, seed):
    code = synth.make_code(N, k, m, seed_graph=300 + m, seed_labels=400 + k)
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, F, seed=seed)
    llr = synth.bpsk_awgn_llr(cw, m, ebn0, code.design_rate, seed=seed + 1)
    return code, enc, cw, llr


def _drain(pool, ncodes, results, max_steps=400):
    for _ in range(max_steps):
        pool.step(2)
        for k in range(ncodes):
            tags, it, st, hd = pool.harvest(k, 4096)
            for i, t in enumerate(tags):
                results[k][int(t)] = (int(it[i]), int(st[i]), hd[i].copy())
        if all(pool.active(k) == 0 for k in range(ncodes)):
            return
    raise AssertionError("pool did not drain")


@pytest.mark.parametrize("tail", ["tail", "full"])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_alone_equals_in_the_mix(prec, tail):
    """tail: steps run the few-frames form (edge-parallel pass) whenever the
    admitted-but-unharvested count allows; full: never (tail threshold 0)."""
    F = 48
    fams = [_family(m, k, N, e, F, seed=10 * i + 1) for i, (_, m, k, N, e) in enumerate(MIX)]
    codes = [D.Code.from_synth(f[0]) for f in fams]
    if tail == "full":
        for c in codes:
            c.set_tuning(tail_frames=0)
    alone = []
    for code, (sc, enc, cw, llr) in zip(codes, fams):
        r = D.decode(code, torch.from_numpy(llr).cuda(), 30, prec=prec, mode="fused")
        alone.append({kk: v.cpu().numpy() for kk, v in r.items()})
    # the mix: slots fewer than frames, admission in three waves while earlier
    # frames are in flight, other codes always present
    pool = D.Pool(codes, [20, 16, 12], prec=prec)
    results = [dict() for _ in codes]
    dev_llr = [torch.from_numpy(f[3]).cuda() for f in fams]
    pending = [0] * len(codes)
    for wave in range(200):
        for k in range(len(codes)):
            if pending[k] < F:
                take = min(7 + 3 * k, F - pending[k])
                got = pool.submit(k, dev_llr[k][pending[k]:pending[k] + take].contiguous(),
                                  np.arange(pending[k], pending[k] + take), 30)
                pending[k] += got
        pool.step(1 + wave % 3)
        for k in range(len(codes)):
            tags, it, st, hd = pool.harvest(k, 4096)
            for i, t in enumerate(tags):
                results[k][int(t)] = (int(it[i]), int(st[i]), hd[i].copy())
        if all(p == F for p in pending) and all(len(r) == F for r in results):
            break
    _drain(pool, len(codes), results)
    for k in range(len(codes)):
        assert len(results[k]) == F
        for f in range(F):
            it, st, hd = results[k][f]
            assert it == alone[k]["iters"][f], (k, f)
            assert st == alone[k]["status"][f], (k, f)
            assert np.array_equal(hd, alone[k]["hard"][f]), (k, f)
    pool.close()
    for c in codes:
        c.close()


def test_pool_slots_and_oracle_results():
    """Admission never exceeds the free slots; harvesting frees them; FP32
    results match the FP64 oracle."""
    sc, enc, cw, llr = _family(6, 6, 60, 2.5, 40, seed=5)
    code = D.Code.from_synth(sc)
    pool = D.Pool([code], [16], prec="fp32")
    dev = torch.from_numpy(llr).cuda()
    assert pool.free_slots(0) == 16
    got = pool.submit(0, dev, np.arange(40), 40)
    assert got == 16 and pool.free_slots(0) == 0
    assert pool.submit(0, dev[16:], np.arange(16, 40), 40) == 0
    results = [dict()]
    done = 16
    for _ in range(400):
        pool.step(3)
        tags, it, st, hd = pool.harvest(0, 64)
        for i, t in enumerate(tags):
            results[0][int(t)] = (int(it[i]), int(st[i]), hd[i].copy())
        if done < 40:
            n = pool.submit(0, dev[done:].contiguous(), np.arange(done, 40), 40)
            done += n
        assert pool.free_slots(0) <= 16
        if done == 40 and len(results[0]) == 40:
            break
    assert len(results[0]) == 40
    tc = TannerCode(sc.M, sc.N, sc.m, sc.row_ptr, sc.col, sc.val, sc.poly)
    ref = odecode(tc, llr, 40)
    same = np.mean([np.array_equal(results[0][f][2], ref.hard[f]) and results[0][f][0] == ref.iters[f]
                    for f in range(40)])
    assert same >= 0.95
    assert pool.free_slots(0) == 16
    pool.close()
    code.close()
