"""Literal FP64 Log-Fourier sum-product decoder (Sec. 3.2) — test infrastructure.

A second CPU implementation, sharing with ``oracle.sp`` only the code
structure, the field arithmetic and the channel pmf, that follows the Log-Fourier SP algorithm step by
step in the signed-log domain.  Tests check it against ``oracle.sp``; the pair
pins the reformulation: the label-map direction, the Gamma map, the
log-convolution of Eq. (6) and the Fourier-domain decisions.

A message entry is a pair (s, l) in GF(2) x [-inf, 0]: Gamma(x) = (sgn(x),
ln|x|) with sgn(0) taken as 0 (the paper leaves it random; a fixed choice keeps
results deterministic).  Products of reals become (XOR, +) on pairs.

Steps (Sec. 3.2):
* INITIALIZATION: Lambda_v^(0)(z) = Gamma(P_v^(0)(z)), P^(0) the Fourier
  transform of p_v^(0); sent to every adjacent check; l := 0.
* CHECK TO VARIABLE: Lambda~_vc(z) = Lambda_vc(H_cv z); Lambda~_cv(z) = sum of
  Lambda~_v'c(z) over v' in V_c minus v (component-wise, k-1 terms);
  Lambda_cv(z) = Lambda~_cv(H_cv^-1 z); l := l + 1.  H_cv is read as M_h^T, the
  transpose of the matrix of x -> h_cv x (the consistent reading of Appendix A:
  the Fourier transform of p(h^-1 x) is P(M_h^T z)).
* VARIABLE TO CHECK: Lambda_vc = Lambda_v^(0) [+] (log-convolution over C_v
  minus c of Lambda_c'v), Eq. (6); then normalised to Lambda_vc(0) = (0, 0), the
  Fourier-domain form of the normalisation P_vc(0) = 1 of Sec. 3.1.
* TENTATIVE DECISION: M_v = Lambda_v^(0) [+] (log-convolution over C_v);
  bit i of x^_v = first entry of M_v(alpha^(i-1)); syndrome bit i of check c =
  first entry of sum over v in V_c of M_v(H_cv alpha^(i-1)).

The log-convolution [+] is evaluated directly over all q^2 pairs as a signed
log-sum-exp: positive and negative terms are summed separately in the log
domain (A, B) and combined as Gamma(e^A - e^B).  ``counts`` tallies the
pairwise log-convolutions (CONV) and component-wise vector additions (ADD) per
node type for comparison with Table 1.
"""
from __future__ import annotations

from collections import Counter
from dataclasses import dataclass

import numpy as np

from .gf import hadamard
from .sp import TannerCode, channel_prior

NEG_INF = -np.inf


def gamma(x: np.ndarray):
    """Gamma(x) = (sgn_GF(2)(x), ln|x|), sgn(0) = 0."""
    x = np.asarray(x, dtype=np.float64)
    s = (x < 0).astype(np.int64)
    with np.errstate(divide="ignore"):
        l = np.log(np.abs(x))
    return s, l


def gamma_inv(s, l):
    return np.where(np.asarray(s) == 1, -1.0, 1.0) * np.exp(l)


def _lse(l: np.ndarray, mask: np.ndarray, axis: int) -> np.ndarray:
    """log sum exp of l over entries where mask is True (-inf if none)."""
    lm = np.where(mask, l, NEG_INF)
    mx = np.max(lm, axis=axis, keepdims=True)
    mx_safe = np.where(np.isfinite(mx), mx, 0.0)
    with np.errstate(divide="ignore"):
        out = np.log(np.sum(np.exp(lm - mx_safe), axis=axis)) + np.squeeze(mx_safe, axis)
    return np.where(np.isfinite(np.squeeze(mx, axis)), out, NEG_INF)


def logconv(s1, l1, s2, l2, xor_table):
    """(lambda1 [+] lambda2)(z) = Gamma( sum_{z1+z2=z} Gamma^-1(lambda1(z1)+lambda2(z2)) ),
    Eq. (6), over all q^2 pairs."""
    # pair (z1, z): z2 = z1 ^ z
    s2p = s2[..., xor_table]                 # [..., z1, z]
    l2p = l2[..., xor_table]
    s = s1[..., :, None] ^ s2p
    l = l1[..., :, None] + l2p
    A = _lse(l, s == 0, axis=-2)             # positive part
    B = _lse(l, s == 1, axis=-2)             # negative part
    big = np.maximum(A, B)
    small = np.minimum(A, B)
    with np.errstate(divide="ignore", invalid="ignore"):
        diff = np.where(np.isfinite(big), small - big, NEG_INF)
        lm = np.where(np.isfinite(big), big + np.log1p(-np.exp(diff)), NEG_INF)
    sign = (B > A).astype(np.int64)          # A == B -> value 0 -> sign 0
    lm = np.where(A == B, NEG_INF, lm)
    return sign, lm


@dataclass
class LFState:
    s: np.ndarray   # [F, E, q] signs
    l: np.ndarray   # [F, E, q] log magnitudes


class LogFourierSP:
    def __init__(self, code: TannerCode):
        self.code = code
        g = code.gf
        q = code.q
        self.H = hadamard(q)
        self.perm = np.stack([g.fourier_perm(h) for h in code.edge_label])        # H_cv z
        self.perm_inv = np.argsort(self.perm, axis=1)                              # H_cv^-1 z
        self.xor_table = np.arange(q)[:, None] ^ np.arange(q)[None, :]
        self.counts = Counter()

    # INITIALIZATION
    def init(self, llr):
        p0 = channel_prior(llr, self.code.m)
        P0 = p0 @ self.H.T
        return gamma(P0)                       # Lambda_v^(0): ([F,N,q], [F,N,q])

    # CHECK TO VARIABLE
    def check_to_var(self, v2c: LFState) -> LFState:
        code = self.code
        F, E, q = v2c.s.shape
        out_s = np.zeros_like(v2c.s)
        out_l = np.zeros_like(v2c.l)
        for c in range(code.M):
            es = np.arange(code.row_ptr[c], code.row_ptr[c + 1])
            # Lambda~_vc(z) = Lambda_vc(H_cv z)
            ts = [v2c.s[:, e, self.perm[e]] for e in es]
            tl = [v2c.l[:, e, self.perm[e]] for e in es]
            for j, e in enumerate(es):
                acc_s = np.zeros((F, q), np.int64)
                acc_l = np.zeros((F, q))
                terms = 0
                for jj in range(len(es)):
                    if jj != j:
                        acc_s = acc_s ^ ts[jj]
                        acc_l = acc_l + tl[jj]
                        terms += 1
                self.counts["check_ADD"] += max(terms - 1, 0)
                # Lambda_cv(z) = Lambda~_cv(H_cv^-1 z)
                out_s[:, e] = acc_s[:, self.perm_inv[e]]
                out_l[:, e] = acc_l[:, self.perm_inv[e]]
        return LFState(out_s, out_l)

    def _fold(self, L0s, L0l, edges, msgs: LFState, skip=None):
        s, l = L0s, L0l
        for e in edges:
            if e == skip:
                continue
            s, l = logconv(s, l, msgs.s[:, e], msgs.l[:, e], self.xor_table)
            self.counts["fold_CONV"] += 1
        return s, l

    # VARIABLE TO CHECK
    def var_to_check(self, L0, c2v: LFState) -> LFState:
        code = self.code
        out_s = np.zeros_like(c2v.s)
        out_l = np.zeros_like(c2v.l)
        for v in range(code.N):
            edges = [e for e in code.var_edges[v] if e < code.E]
            for e in edges:
                before = self.counts["fold_CONV"]
                s, l = self._fold(L0[0][:, v], L0[1][:, v], edges, c2v, skip=e)
                self.counts["var_CONV"] += self.counts["fold_CONV"] - before
                # normalise Lambda_vc(0) = (0, 0)
                if np.any(s[:, 0] != 0):
                    raise FloatingPointError("V2C Fourier value at z=0 must be positive")
                out_s[:, e] = s
                out_l[:, e] = l - l[:, :1]
        return LFState(out_s, out_l)

    # TENTATIVE DECISION
    def tentative(self, L0, c2v: LFState):
        code = self.code
        F = c2v.s.shape[0]
        m = code.m
        Ms = np.zeros((F, code.N, code.q), np.int64)
        Ml = np.zeros((F, code.N, code.q))
        for v in range(code.N):
            edges = [e for e in code.var_edges[v] if e < code.E]
            before = self.counts["fold_CONV"]
            Ms[:, v], Ml[:, v] = self._fold(L0[0][:, v], L0[1][:, v], edges, c2v)
            self.counts["tent_CONV"] += self.counts["fold_CONV"] - before
        # x^_{v,i} = first entry of M_v(alpha^(i-1))
        bits = Ms[:, :, 1 << np.arange(m)]
        hard = (bits << np.arange(m)).sum(-1)
        # s^_{c,i} = first entry of sum_{v in V_c} M_v(H_cv alpha^(i-1))
        fs = np.zeros((F, code.M), np.int64)
        ds = np.zeros((F, code.M), np.int64)
        for e in range(code.E):
            c, v, h = code.edge_check[e], code.edge_var[e], code.edge_label[e]
            pts = self.perm[e][1 << np.arange(m)]
            fs[:, c] ^= (Ms[:, v, pts] << np.arange(m)).sum(-1)
            ds[:, c] ^= code.gf.mul(h, hard[:, v])
        return Ms, Ml, hard, fs, ds

    def run(self, llr, rounds: int):
        """Rounds 1..rounds without stopping; returns per-round c2v, v2c states
        and decisions (hard, fourier syndrome, direct syndrome)."""
        code = self.code
        L0 = self.init(llr)
        v2c = LFState(L0[0][:, code.edge_var], L0[1][:, code.edge_var])
        hist = []
        for _ in range(rounds):
            c2v = self.check_to_var(v2c)
            v2c = self.var_to_check(L0, c2v)
            _, _, hard, fs, ds = self.tentative(L0, c2v)
            hist.append((c2v, v2c, hard, fs, ds))
        return L0, hist
