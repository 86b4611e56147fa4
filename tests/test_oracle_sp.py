"""Pins of the FP64 sum-product oracle and the literal Log-Fourier reference
against brute force, textbook binary BP, closed forms and invariants."""
import itertools

import numpy as np
import pytest

from oracle.gf import hadamard
from oracle.lfsp import LogFourierSP, gamma_inv
from oracle.sp import (TannerCode, channel_prior, check_to_var, decode, fourier,
                       run_rounds, tentative, var_to_check)
from paper_1008_4370_amd import synth


def _tc(code):
    return TannerCode(code.M, code.N, code.m, code.row_ptr, code.col, code.val, code.poly)


def _prior_bf(L):
    """Per-symbol pmf from bit LLRs, written out for the brute-force checks."""
    m = L.shape[-1]
    q = 1 << m
    out = np.ones(L.shape[:-1] + (q,))
    for x in range(q):
        for i in range(m):
            s = 1.0 if ((x >> i) & 1) == 0 else -1.0
            out[..., x] *= 1.0 / (1.0 + np.exp(-s * L[..., i]))
    return out


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,k", [(2, 3), (3, 4), (4, 3)])
def test_single_check_extrinsic_bruteforce(m, k):
    """Eq. (1) against enumeration of the other k-1 symbols of one check."""
    rng = np.random.default_rng(7 + m)
    q = 1 << m
    labels = rng.integers(1, q, k)
    code = TannerCode(1, k, m, [0, k], np.arange(k), labels)
    f = synth._Field(m, synth.default_poly(m))
    v2c = rng.random((2, k, q))
    v2c /= v2c.sum(-1, keepdims=True)
    c2v = check_to_var(code, v2c)
    for j in range(k):
        bf = np.zeros((2, q))
        others = [jj for jj in range(k) if jj != j]
        for assign in itertools.product(range(q), repeat=k - 1):
            acc = 0
            w = np.ones(2)
            for jj, xj in zip(others, assign):
                acc ^= int(f.mul(labels[jj], xj))
                w = w * v2c[:, jj, xj]
            xj_out = int(f.mul(f.inv(labels[j]), acc)) if acc else 0
            bf[:, xj_out] += w
        assert np.allclose(c2v[:, j], bf, atol=1e-13), j


@pytest.mark.parametrize("m,nchk,seed", [(2, 3, 1), (2, 4, 2), (3, 3, 3), (1, 5, 4), (4, 2, 5)])
def test_tree_posteriors_equal_bruteforce_marginals(m, nchk, seed):
    """On a cycle-free Tanner graph SP yields the exact symbol marginals
    (Sec. 2.1: symbol MAP on trees)."""
    code = synth.make_tree_code(nchk, m, seed)
    enc = synth.Encoder(code)
    q = 1 << m
    assert q ** enc.K <= 20000
    rng = np.random.default_rng(100 + seed)
    F = 3
    L = rng.normal(0.5, 2.0, (F, code.N, m))
    p0 = _prior_bf(L)
    infos = np.array(list(itertools.product(range(q), repeat=enc.K)))
    cws = enc.encode(infos)                                   # all codewords
    assert np.all(enc.syndrome(cws) == 0)
    tc = _tc(code)
    rounds = 2 * nchk + 2
    _, _, decs = run_rounds(tc, L, rounds)
    post = decs[-1].post
    for f in range(F):
        w = np.prod(p0[f, np.arange(code.N)[None, :], cws], axis=1)   # [ncw]
        for v in range(code.N):
            marg = np.bincount(cws[:, v], weights=w, minlength=q)
            marg /= marg.sum()
            assert np.allclose(post[f, v], marg, atol=1e-12), (f, v)


def test_binary_case_is_textbook_tanh_bp():
    """m = 1: the decoder is binary belief propagation with the tanh rule
    (the method applies to binary codes, Sec. 1)."""
    code = synth.make_code(24, 4, 1, seed_graph=5, seed_labels=6)
    tc = _tc(code)
    rng = np.random.default_rng(9)
    L = rng.normal(1.0, 1.5, (4, code.N, 1))
    R = 5
    _, _, decs = run_rounds(tc, L, R)
    # textbook LLR-domain BP
    E = tc.E
    Lv = L[..., 0]
    Lvc = Lv[:, tc.edge_var].copy()
    for _ in range(R):
        Lcv = np.zeros_like(Lvc)
        for c in range(tc.M):
            es = range(tc.row_ptr[c], tc.row_ptr[c + 1])
            for e in es:
                prod = np.ones(Lv.shape[0])
                for e2 in es:
                    if e2 != e:
                        prod = prod * np.tanh(Lvc[:, e2] / 2)
                Lcv[:, e] = 2 * np.arctanh(prod)
        tot = Lv.copy()
        for e in range(E):
            tot[:, tc.edge_var[e]] += Lcv[:, e]
        Lvc = tot[:, tc.edge_var] - Lcv
    post = decs[-1].post
    llr_oracle = np.log(post[..., 0] / post[..., 1])
    assert np.allclose(llr_oracle, tot, atol=1e-8)


def _gf4_batch(frames=40):
    return synth.make_batch("gf4_n96", frames=frames)


def test_noiseless_decodes_in_one_round():
    b = _gf4_batch(8)
    bits = (b.cw[..., None] >> np.arange(b.code.m)) & 1
    L = 40.0 * (1 - 2 * bits)
    r = decode(_tc(b.code), L, 10)
    assert np.all(r.iters == 1) and np.all(r.converged)
    assert np.array_equal(r.hard, b.cw)


def test_zero_llr_gives_uniform_posteriors_and_zero_word():
    b = _gf4_batch(3)
    L = np.zeros_like(b.llr, dtype=np.float64)
    r = decode(_tc(b.code), L, 10)
    assert np.allclose(r.post, 1.0 / b.code.q)
    assert np.all(r.hard == 0) and np.all(r.iters == 1) and np.all(r.converged)


def test_codeword_shift_symmetry():
    """Flipping the channel LLR signs on the bits of a codeword c maps every
    decision x^ to x^ + c (the decoder is symmetric under codeword shifts)."""
    b = _gf4_batch(30)
    tc = _tc(b.code)
    c = synth.random_codewords(b.enc, 1, seed=77)[0]
    flip = 1 - 2 * ((c[None, :, None] >> np.arange(b.code.m)) & 1)
    r1 = decode(tc, b.llr, 30)
    r2 = decode(tc, b.llr * flip, 30)
    assert np.array_equal(r1.iters, r2.iters)
    assert np.array_equal(r1.converged, r2.converged)
    assert np.array_equal(r1.hard ^ c[None, :].astype(np.uint8), r2.hard)


def test_normalisation_by_p0_gives_the_same_output():
    """Sec. 2.1: normalising V2C messages by p_vc(0) instead of their sum does not
    change the decoding output."""
    b = _gf4_batch(10)
    tc = _tc(b.code)
    L = b.llr.astype(np.float64)
    p0 = channel_prior(L, tc.m)
    v2c_a = p0[:, tc.edge_var]
    v2c_b = v2c_a / v2c_a[..., :1]
    for _ in range(6):
        c2v_a = check_to_var(tc, v2c_a)
        c2v_b = check_to_var(tc, v2c_b)
        da, db = tentative(tc, p0, c2v_a), tentative(tc, p0, c2v_b)
        assert np.array_equal(da.hard, db.hard)
        assert np.allclose(da.post, db.post, atol=1e-12)
        v2c_a = var_to_check(tc, p0, c2v_a)
        v2c_b = var_to_check(tc, p0, c2v_b)
        v2c_b = v2c_b / v2c_b[..., :1]


def test_map_bit_identity_and_symbol_map():
    """Sec. 3.1: Q_v(alpha^(i-1)) = q_{v,i}(0) - q_{v,i}(1); bitwise and symbol MAP
    coincide when max_x q_v(x) > 1/2."""
    b = _gf4_batch(20)
    tc = _tc(b.code)
    _, _, decs = run_rounds(tc, b.llr, 3)
    d = decs[-1]
    Q = fourier(d.post, hadamard(tc.q))
    assert np.allclose(Q[..., 1 << np.arange(tc.m)], d.qbits, atol=1e-14)
    conf = d.post.max(-1) > 0.5
    assert np.array_equal(d.hard[conf], d.symmap[conf])


def test_fourier_syndrome_can_differ_from_direct_syndrome():
    """The paper's Fourier syndrome is H x^ only for confident posteriors: a GF(4)
    posterior with q(00)=.40, q(10)=.25, q(11)=.35 (bits x_1 x_2 as integer
    bit0 bit1) has Q(e1)>0, Q(e2)<0 but Q(e1+e2)>0 (parity 0), while
    x^_1 + x^_2 = 1."""
    q = np.zeros(4)
    q[0b00], q[0b10], q[0b11], q[0b01] = 0.40, 0.25, 0.35, 0.0
    Q = fourier(q[None], hadamard(4))[0]
    assert Q[1] > 0 and Q[2] < 0 and Q[3] > 0
    x1, x2 = int(Q[1] < 0), int(Q[2] < 0)
    assert (x1 ^ x2) != int(Q[3] < 0)


def test_syndromes_and_stopping_rule():
    b = _gf4_batch(60)
    tc = _tc(b.code)
    r = decode(tc, b.llr, 20)
    assert np.array_equal(r.synd, b.enc.syndrome(r.hard.astype(np.int64)))
    assert np.all((r.iters >= 1) & (r.iters <= 20))
    assert np.all(r.synd[r.converged] == 0) and np.all(r.fsynd[r.converged] == 0)
    assert np.all(r.iters[~r.converged] == 20)
    # Fourier syndrome equals H x^ whenever every posterior is confident
    conf = (r.post.max(-1) > 0.5).all(-1)
    assert conf.sum() > 10
    assert np.array_equal(r.fsynd[conf], r.synd[conf])
    r1 = decode(tc, b.llr, 1)
    assert np.all(r1.iters == 1)


@pytest.mark.parametrize("m,N,k", [(2, 16, 4), (3, 12, 3), (4, 12, 4)])
def test_log_fourier_reference_matches_sp(m, N, k):
    """Sec. 3: the Log-Fourier SP outputs the same results as SP; messages agree
    in the linear Fourier domain to FP64 rounding."""
    code = synth.make_code(N, k, m, seed_graph=11 * m, seed_labels=13 * m)
    tc = _tc(code)
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, 3, seed=m)
    L = synth.bpsk_awgn_llr(cw, m, 1.5, code.design_rate, seed=m, dtype=np.float64)
    lf = LogFourierSP(tc)
    _, hist = lf.run(L, 4)
    c2vs, v2cs, decs = run_rounds(tc, L, 4)
    H = hadamard(tc.q)
    for t in range(4):
        c2v_lf, v2c_lf, hard, fs, ds = hist[t]
        assert np.abs(gamma_inv(c2v_lf.s, c2v_lf.l) - fourier(c2vs[t], H)).max() < 1e-10
        assert np.abs(gamma_inv(v2c_lf.s, v2c_lf.l) - fourier(v2cs[t], H)).max() < 1e-10
        assert np.array_equal(hard, decs[t].hard)
        assert np.array_equal(fs, decs[t].fsynd)
        assert np.array_equal(ds, decs[t].synd)


def test_table1_operation_counts():
    """Table 1, Log-Fourier SP row, per round of a (2,k) code: each variable node
    does two 2-fold CONVs (V2C) and one 3-fold CONV (= 2 pairwise) for the
    tentative decision; each check does k (k-1)-term ADDs (k-2 pairwise each)."""
    code = synth.make_code(12, 4, 2, seed_graph=3, seed_labels=4)
    tc = _tc(code)
    lf = LogFourierSP(tc)
    L = np.random.default_rng(0).normal(1, 1, (1, code.N, 2))
    lf.run(L, 1)
    deg = np.diff(code.row_ptr)
    assert lf.counts["var_CONV"] == 2 * code.N
    assert lf.counts["tent_CONV"] == 2 * code.N
    assert lf.counts["check_ADD"] == int(np.sum(deg * (deg - 2)))


@pytest.mark.parametrize("m,nchk,seed", [(2, 3, 11), (3, 3, 12), (2, 4, 13)])
def test_symbol_prior_input_tree_marginals(m, nchk, seed):
    """Channel input given as symbol priors Pr(X_v = x | y_v) (Sec. 2.1) that do
    not factor over bits: on a cycle-free graph the posteriors are the exact
    marginals of prod_v p0_v(x_v) over the codewords."""
    code = synth.make_tree_code(nchk, m, seed)
    enc = synth.Encoder(code)
    q = 1 << m
    rng = np.random.default_rng(200 + seed)
    F = 2
    p0 = rng.random((F, code.N, q)) ** 3 + 1e-3          # arbitrary positive, unnormalised
    infos = np.array(list(itertools.product(range(q), repeat=enc.K)))
    cws = enc.encode(infos)
    tc = _tc(code)
    res = decode(tc, None, 2 * nchk + 2, early_stop=False, prior=p0)
    pn = p0 / p0.sum(-1, keepdims=True)
    for f in range(F):
        w = np.prod(pn[f, np.arange(code.N)[None, :], cws], axis=1)
        for v in range(code.N):
            marg = np.bincount(cws[:, v], weights=w, minlength=q)
            assert np.allclose(res.post[f, v], marg / marg.sum(), atol=1e-12), (f, v)


def test_symbol_prior_input_equals_llr_input():
    """The BPSK prior passed as symbol priors decodes exactly like the LLRs."""
    code = synth.make_code(40, 4, 3, seed_graph=31, seed_labels=32)
    tc = _tc(code)
    enc = synth.Encoder(code)
    cw = synth.random_codewords(enc, 6, seed=33)
    llr = synth.bpsk_awgn_llr(cw, 3, 2.0, code.design_rate, seed=34).astype(np.float64)
    a = decode(tc, llr, 30)
    b = decode(tc, None, 30, prior=channel_prior(llr, 3))
    assert np.array_equal(a.hard, b.hard) and np.array_equal(a.iters, b.iters)
    assert np.allclose(a.post, b.post, atol=1e-12)
