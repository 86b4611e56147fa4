"""Probability-domain sum-product (SP) decoder in FP64 — THE parity oracle.

Test infrastructure only (see ``oracle/__init__``).  This is the plain
definition that the Log-Fourier SP method reaches exactly up to rounding: the
paper designs the Fourier SP to give the same decoding output as SP and Log-SP
(Sec. 3, introduction) and Log-SP to equal SP (end of Sec. 2.2).

Every step follows the paper's order and notation:

* INITIALIZATION (Sec. 2.1): p_v^(0)(x) = Pr(X_v = x | Y_v = y_v); every
  variable sends p_vc = p_v^(0); l := 0.  For the BPSK channel the bits of a
  symbol are independent given y, so p_v^(0)(x) = prod_i Pr(b_i = x_i | y_i)
  with Pr(b = 0 | y) = sigma(L), L = ln Pr(b=0|y)/Pr(b=1|y), sigma(t) =
  1/(1+e^-t).
* CHECK TO VARIABLE (Sec. 2.1, Eq. (1)): p~_vc(x) = p_vc(h_cv^-1 x);
  p~_cv = XOR-convolution of p~_v'c over v' in V_c minus v, each convolution
  evaluated directly in O(q^2); p_cv(x) = p~_cv(h_cv x); then l := l + 1.
* VARIABLE TO CHECK (Sec. 2.1): p_vc(x) = p_v^(0)(x) prod_{c' in C_v minus c}
  p_c'v(x), normalised to sum 1.
* TENTATIVE DECISION (Sec. 2.1 and the bitwise-MAP / Fourier-syndrome rules of
  Sec. 3.1, Eq. (5), repeated for the Log-Fourier SP in Sec. 3.2):
  q_v(x) = p_v^(0)(x) prod_{c in C_v} p_cv(x) (normalised);
  bit i of x^_v is 1 iff the marginal q_{v,i}(1) > q_{v,i}(0) (a tie gives 0,
  a deterministic choice where the paper leaves ties to a random one);
  direct syndrome s_c = sum_{v in V_c} h_cv x^_v;
  Fourier syndrome bit i of check c = XOR over v in V_c of [Q_v(M_h^T e_i) < 0]
  with Q_v the Fourier transform of q_v and h = h_cv.
* STOP (Sec. 2, step 4): the decoder stops at the first l whose decision passes
  the codeword test and reports FAIL when l reaches max_iter.  The codeword
  test requires BOTH syndromes to be zero: the Fourier syndrome is the paper's
  test, and the direct syndrome guards the cases where the Fourier syndrome
  differs from H x^ (it can, when a posterior has max_x q_v(x) <= 1/2).

Codes may have any row and column weights (the paper notes the extension to
irregular codes is straightforward, Sec. 2); the tree tests rely on this.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .gf import GF, hadamard


class TannerCode:
    """The code {x : Hx = 0} of an M x N parity-check matrix over GF(2^m)
    (Sec. 2), given in compressed-row form.  Edge e is the e-th nonzero of H in
    row-major order: (check, variable, label h_cv)."""

    def __init__(self, M, N, m, row_ptr, col, val, poly=None):
        self.gf = GF(m, poly)
        self.M, self.N, self.m, self.q = int(M), int(N), int(m), 1 << int(m)
        self.row_ptr = np.asarray(row_ptr, dtype=np.int64)
        self.col = np.asarray(col, dtype=np.int64)
        self.val = np.asarray(val, dtype=np.int64)
        self.E = len(self.col)
        if self.row_ptr[-1] != self.E or len(self.row_ptr) != self.M + 1:
            raise ValueError("bad row_ptr")
        if np.any(self.val <= 0) or np.any(self.val >= self.q):
            raise ValueError("labels must be nonzero field elements")
        self.edge_check = np.repeat(np.arange(self.M), np.diff(self.row_ptr))
        self.edge_var = self.col.copy()
        self.edge_label = self.val.copy()
        deg_c = np.diff(self.row_ptr)
        self.kmax = int(deg_c.max()) if self.M else 0
        # V_c as a padded table of edge ids (padding = E, the identity slot)
        self.check_edges = np.full((self.M, max(self.kmax, 1)), self.E, dtype=np.int64)
        for c in range(self.M):
            es = np.arange(self.row_ptr[c], self.row_ptr[c + 1])
            self.check_edges[c, : len(es)] = es
        # C_v as a padded table of edge ids
        deg_v = np.bincount(self.col, minlength=self.N)
        self.dmax = int(deg_v.max()) if self.N else 0
        self.var_edges = np.full((self.N, max(self.dmax, 1)), self.E, dtype=np.int64)
        fill = np.zeros(self.N, dtype=np.int64)
        for e in range(self.E):
            v = self.col[e]
            self.var_edges[v, fill[v]] = e
            fill[v] += 1
        # per-edge index maps of the label permutations of Eq. (1)
        g = self.gf
        xs = np.arange(self.q)
        self.idx_hinv = np.stack([g.mul(g.inv(h), xs) for h in self.edge_label]) if self.E else np.zeros((0, self.q), np.int64)
        self.idx_h = np.stack([g.mul(h, xs) for h in self.edge_label]) if self.E else np.zeros((0, self.q), np.int64)
        # Fourier-syndrome evaluation points M_h^T e_i per edge (Sec. 3.1)
        self.fsyn_pts = np.stack([g.fourier_perm(h)[1 << np.arange(self.m)] for h in self.edge_label]) if self.E else np.zeros((0, self.m), np.int64)
        self.H = hadamard(self.q)
        self.xor_table = np.arange(self.q)[:, None] ^ np.arange(self.q)[None, :]


# ---------------------------------------------------------------------------
# message-domain primitives
# ---------------------------------------------------------------------------
def sigma(t):
    return 1.0 / (1.0 + np.exp(-t))


def channel_prior(llr: np.ndarray, m: int) -> np.ndarray:
    """p_v^(0)(x) = prod_i Pr(b_i = x_i | y) for BPSK LLRs [..., m] (INITIALIZATION,
    Sec. 2.1); bit i of the integer x is x_{i+1} (Sec. 2)."""
    llr = np.asarray(llr, dtype=np.float64)
    q = 1 << m
    p = np.ones(llr.shape[:-1] + (q,), dtype=np.float64)
    for x in range(q):
        for i in range(m):
            b = (x >> i) & 1
            p[..., x] *= sigma(llr[..., i] if b == 0 else -llr[..., i])
    return p


def xor_conv(p1: np.ndarray, p2: np.ndarray, xor_table: np.ndarray) -> np.ndarray:
    """(p1 (x) p2)(x) = sum_{x1 + x2 = x} p1(x1) p2(x2), evaluated directly
    (O(q^2), the definition below Eq. (1))."""
    # p2[..., x1 ^ x] as a [..., x1, x] matrix
    return np.einsum("...a,...ax->...x", p1, p2[..., xor_table])


def fourier(p: np.ndarray, H: np.ndarray) -> np.ndarray:
    """P(z) = sum_x p(x) (-1)^(z.x) (Sec. 2.1)."""
    return p @ H.T


# ---------------------------------------------------------------------------
# the four steps
# ---------------------------------------------------------------------------
def check_to_var(code: TannerCode, v2c: np.ndarray) -> np.ndarray:
    """CHECK TO VARIABLE, Eq. (1).  v2c: [F, E, q] -> c2v: [F, E, q]."""
    F, q = v2c.shape[0], code.q
    # p~_vc(x) = p_vc(h^-1 x)
    pt = np.take_along_axis(v2c, code.idx_hinv[None, :, :].repeat(F, 0), axis=2)
    delta = np.zeros((F, 1, q))
    delta[:, 0, 0] = 1.0                      # identity of the XOR convolution
    pt = np.concatenate([pt, delta], axis=1)  # slot E = identity (padding)
    ce = code.check_edges                     # [M, kmax]
    k = ce.shape[1]
    msgs = pt[:, ce, :]                       # [F, M, kmax, q]
    c2v = np.zeros((F, code.E + 1, q))
    for j in range(k):
        acc = np.broadcast_to(delta, (F, code.M, q)).copy()
        for jj in range(k):
            if jj != j:
                acc = xor_conv(acc, msgs[:, :, jj, :], code.xor_table)
        c2v[:, ce[:, j], :] = acc
    c2v = c2v[:, : code.E, :]
    # p_cv(x) = p~_cv(h x)
    return np.take_along_axis(c2v, code.idx_h[None, :, :].repeat(F, 0), axis=2)


def _var_products(code: TannerCode, p0: np.ndarray, c2v: np.ndarray):
    """Products p_v^(0) * prod over C_v of incoming messages, with one slot left
    out (extrinsic, per edge) and with none left out (posterior)."""
    F, q = c2v.shape[0], code.q
    ones = np.ones((F, 1, q))
    msg = np.concatenate([c2v, ones], axis=1)   # slot E = 1 (padding)
    ve = code.var_edges                        # [N, dmax]
    inc = msg[:, ve, :]                        # [F, N, dmax, q]
    post = p0.copy()
    for s in range(ve.shape[1]):
        post = post * inc[:, :, s, :]
    ext = np.zeros((F, code.E + 1, q))
    for s in range(ve.shape[1]):
        prod = p0.copy()
        for ss in range(ve.shape[1]):
            if ss != s:
                prod = prod * inc[:, :, ss, :]
        ext[:, ve[:, s], :] = prod
    return ext[:, : code.E, :], post


def var_to_check(code: TannerCode, p0: np.ndarray, c2v: np.ndarray) -> np.ndarray:
    """VARIABLE TO CHECK (Sec. 2.1): p_vc = p0 * prod_{c' != c} p_c'v, normalised
    to sum 1."""
    ext, _ = _var_products(code, p0, c2v)
    return ext / ext.sum(axis=2, keepdims=True)


@dataclass
class Decision:
    post: np.ndarray     # [F, N, q] normalised posterior q_v
    hard: np.ndarray     # [F, N]    bitwise-MAP symbols (integers)
    symmap: np.ndarray   # [F, N]    symbol-MAP argmax_x q_v(x) (smallest x on ties)
    synd: np.ndarray     # [F, M]    direct syndrome symbols s_c = sum h_cv x^_v
    fsynd: np.ndarray    # [F, M]    Fourier syndrome words (bit i = s^_{c,i+1})
    qbits: np.ndarray    # [F, N, m] Q_v(alpha^(i-1)) = q_{v,i}(0) - q_{v,i}(1)


def tentative(code: TannerCode, p0: np.ndarray, c2v: np.ndarray) -> Decision:
    """TENTATIVE DECISION with the bitwise-MAP rule and both syndromes."""
    g, m, q = code.gf, code.m, code.q
    _, post = _var_products(code, p0, c2v)
    post = post / post.sum(axis=2, keepdims=True)
    xs = np.arange(q)
    # bit marginals q_{v,i}(0) - q_{v,i}(1)
    qbits = np.stack([post[..., ((xs >> i) & 1) == 0].sum(-1) - post[..., ((xs >> i) & 1) == 1].sum(-1)
                      for i in range(m)], axis=-1)
    bits = (qbits < 0).astype(np.int64)                 # tie (== 0) -> 0
    hard = (bits << np.arange(m)).sum(-1)
    symmap = post.argmax(-1)
    # direct syndrome
    contrib = g.mul(code.edge_label[None, :], hard[:, code.edge_var])  # [F, E]
    F = post.shape[0]
    synd = np.zeros((F, code.M), dtype=np.int64)
    for e in range(code.E):
        synd[:, code.edge_check[e]] ^= contrib[:, e]
    # Fourier syndrome from Q_v at M_h^T e_i
    Q = fourier(post, code.H)                           # [F, N, q]
    fs = np.zeros((F, code.M), dtype=np.int64)
    for e in range(code.E):
        vals = Q[:, code.edge_var[e], code.fsyn_pts[e]]  # [F, m]
        word = ((vals < 0).astype(np.int64) << np.arange(m)).sum(-1)
        fs[:, code.edge_check[e]] ^= word
    return Decision(post, hard, symmap, synd, fs, qbits)


# ---------------------------------------------------------------------------
# driver
# ---------------------------------------------------------------------------
@dataclass
class Result:
    hard: np.ndarray        # [F, N] uint8 bitwise-MAP symbols at the stopping round
    symmap: np.ndarray      # [F, N] symbol-MAP symbols at the stopping round
    synd: np.ndarray        # [F, M] direct syndrome of `hard`
    fsynd: np.ndarray       # [F, M] Fourier syndrome words at the stopping round
    iters: np.ndarray       # [F] l at which the decoder stopped (1..max_iter)
    converged: np.ndarray   # [F] bool: stopped on a passed codeword test
    mismatch: np.ndarray    # [F] bool: Fourier and direct syndromes differed at some round
    post: np.ndarray        # [F, N, q] posterior at the stopping round
    qbits: np.ndarray       # [F, N, m]


def decode(code: TannerCode, llr: np.ndarray, max_iter: int, early_stop: bool = True,
           chunk: int = 64, prior: np.ndarray | None = None) -> Result:
    """Flooding SP decoding of every frame of llr [F, N, m] (Sec. 2, steps 1-4).
    With prior [F, N, q] (llr ignored, may be None) the channel input is the
    symbol prior Pr(X_v = x | y_v) itself (INITIALIZATION, Sec. 2.1),
    normalised per symbol."""
    if prior is not None:
        src = np.asarray(prior, dtype=np.float64)
        src = src / src.sum(axis=-1, keepdims=True)
    else:
        src = np.asarray(llr, dtype=np.float64)
    F = src.shape[0]
    parts = [_decode_chunk(code, src[i:i + chunk], max_iter, early_stop, prior is not None)
             for i in range(0, F, chunk)]
    if not parts:
        parts = [_decode_chunk(code, src, max_iter, early_stop, prior is not None)]
    return Result(*[np.concatenate([getattr(p, f) for p in parts]) for f in Result.__dataclass_fields__])


def _decode_chunk(code, src, max_iter, early_stop, is_prior=False):
    F, N, M, q, m = src.shape[0], code.N, code.M, code.q, code.m
    p0 = src if is_prior else channel_prior(src, m)
    res = Result(hard=np.zeros((F, N), np.int64), symmap=np.zeros((F, N), np.int64),
                 synd=np.zeros((F, M), np.int64), fsynd=np.zeros((F, M), np.int64),
                 iters=np.zeros(F, np.int64), converged=np.zeros(F, bool),
                 mismatch=np.zeros(F, bool), post=np.zeros((F, N, q)), qbits=np.zeros((F, N, m)))
    if max_iter < 1:
        raise ValueError("max_iter must be >= 1")
    act = np.arange(F)
    v2c = p0[:, code.edge_var, :]            # INITIALIZATION: p_vc = p_v^(0); l = 0
    for ell in range(1, max_iter + 1):
        if len(act) == 0:
            break
        c2v = check_to_var(code, v2c)        # CHECK TO VARIABLE; l := l + 1
        v2c = var_to_check(code, p0[act], c2v)
        d = tentative(code, p0[act], c2v)
        res.hard[act], res.symmap[act] = d.hard, d.symmap
        res.synd[act], res.fsynd[act] = d.synd, d.fsynd
        res.post[act], res.qbits[act] = d.post, d.qbits
        res.iters[act] = ell
        res.mismatch[act] |= np.any(d.synd != d.fsynd, axis=1)
        ok = np.all(d.synd == 0, axis=1) & np.all(d.fsynd == 0, axis=1)
        res.converged[act] = ok
        if early_stop:
            keep = ~ok
            act, v2c = act[keep], v2c[keep]
    res.hard = res.hard.astype(np.uint8)
    return res


def run_rounds(code: TannerCode, llr: np.ndarray, rounds: int):
    """Messages of rounds 1..rounds without stopping: lists of c2v and v2c
    arrays (prob domain, variable coordinates) and the decisions per round."""
    llr = np.asarray(llr, dtype=np.float64)
    p0 = channel_prior(llr, code.m)
    v2c = p0[:, code.edge_var, :]
    out_c2v, out_v2c, out_dec = [], [], []
    for _ in range(rounds):
        c2v = check_to_var(code, v2c)
        v2c = var_to_check(code, p0, c2v)
        out_c2v.append(c2v)
        out_v2c.append(v2c)
        out_dec.append(tentative(code, p0, c2v))
    return out_c2v, out_v2c, out_dec
