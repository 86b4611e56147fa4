"""Seeded synthetic inputs: codes, codewords and BPSK/AWGN channel LLRs.

This module is shared by the tests, the benchmark and the HIP decoder's users.
It holds none of the decoder's arithmetic: it draws (2,k) Tanner graphs from a
configuration model, labels them, builds a systematic encoder by Gaussian
elimination over GF(2^m) and simulates BPSK over AWGN.  Its small field
arithmetic exists only to encode.

Conventions (the paper fixes none of these; it has no channel model):
* symbol x <-> bits (x_1..x_m), x_i = bit (i-1) of the integer (Sec. 2);
* BPSK: bit 0 -> +1, bit 1 -> -1; y = s + sigma * n; LLR L = 2 y / sigma^2 =
  ln Pr(b=0|y) / Pr(b=1|y); LLR array [F, N, m], bit i of symbol v at [f, v, i];
* Eb/N0 per information bit with the design rate R = 1 - M/N:
  sigma^2 = 1 / (2 R 10^(EbN0/10)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_POLY = {1: 0b11, 2: 0b111, 3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011,
         7: 0b10001001, 8: 0b100011101}


def default_poly(m: int) -> int:
    return _POLY[m]


class _Field:
    """Minimal GF(2^m) for encoding (log/antilog tables)."""

    def __init__(self, m: int, poly: int):
        self.q = q = 1 << m
        self.exp = np.zeros(2 * q, dtype=np.int64)
        self.log = np.zeros(q, dtype=np.int64)
        x = 1
        for i in range(q - 1):
            self.exp[i] = x
            self.log[x] = i
            x <<= 1
            if x & q:
                x ^= poly
        for i in range(q - 1, 2 * q):
            self.exp[i] = self.exp[i - (q - 1)]

    def mul(self, a, b):
        a = np.asarray(a, dtype=np.int64)
        b = np.asarray(b, dtype=np.int64)
        r = self.exp[(self.log[a] + self.log[b]) % (self.q - 1)]
        return np.where((a == 0) | (b == 0), 0, r)

    def inv(self, a):
        return self.exp[(self.q - 1 - self.log[a]) % (self.q - 1)]


@dataclass
class Code:
    """An M x N parity-check matrix over GF(2^m) in compressed-row form."""
    M: int
    N: int
    m: int
    row_ptr: np.ndarray     # int32 [M+1]
    col: np.ndarray         # int32 [E]
    val: np.ndarray         # uint16 [E], labels in 1..q-1
    poly: int
    seeds: dict = field(default_factory=dict)

    @property
    def q(self):
        return 1 << self.m

    @property
    def E(self):
        return len(self.col)

    @property
    def design_rate(self):
        return 1.0 - self.M / self.N

    def dense(self) -> np.ndarray:
        H = np.zeros((self.M, self.N), dtype=np.int64)
        for c in range(self.M):
            for e in range(self.row_ptr[c], self.row_ptr[c + 1]):
                H[c, self.col[e]] = self.val[e]
        return H


def check_degrees(N: int, k: int, j: int = 2, M: int | None = None) -> np.ndarray:
    """Near-regular check degrees: M = round(jN/k) checks whose degrees differ by
    at most one and sum to jN."""
    if M is None:
        M = int(round(j * N / k))
    base, extra = divmod(j * N, M)
    deg = np.full(M, base, dtype=np.int64)
    deg[:extra] += 1
    return deg


def irregular_var_degrees(N: int, dist: dict, seed: int = 1005) -> np.ndarray:
    """Column weights for N variables: round(N * fraction) of each weight in
    `dist` ({weight: fraction}, the largest fraction absorbing the rounding),
    in a seeded random order."""
    ws = sorted(dist)
    counts = {w: int(round(N * dist[w])) for w in ws}
    top = max(ws, key=lambda w: dist[w])
    counts[top] += N - sum(counts.values())
    deg = np.concatenate([np.full(counts[w], w, dtype=np.int64) for w in ws])
    return np.random.default_rng(seed).permutation(deg)


def make_code(N: int, k: int, m: int, seed_graph: int = 1001, seed_labels: int = 1002,
              j: int = 2, M: int | None = None, poly: int | None = None,
              max_retries: int = 200, var_degrees: np.ndarray | None = None) -> Code:
    """Seeded configuration-model (j, k) Tanner graph without double edges and
    with labels uniform on the nonzero field elements.  With var_degrees the
    column weights are those (an irregular code); the checks stay near-regular
    with M = round(E / k) unless M is given."""
    rng = np.random.default_rng(seed_graph)
    if var_degrees is None:
        deg_c = check_degrees(N, k, j, M)
        var_sock = np.repeat(np.arange(N), j)
    else:
        var_degrees = np.asarray(var_degrees, dtype=np.int64)
        E = int(var_degrees.sum())
        Mi = int(round(E / k)) if M is None else M
        base, extra = divmod(E, Mi)
        deg_c = np.full(Mi, base, dtype=np.int64)
        deg_c[:extra] += 1
        var_sock = np.repeat(np.arange(N), var_degrees)
    M = len(deg_c)
    chk_sock = np.repeat(np.arange(M), deg_c)
    perm = None
    for _ in range(max_retries):
        p = rng.permutation(len(var_sock))
        if not _has_double(chk_sock, var_sock[p], M, N):
            perm = p
            break
    if perm is None:
        perm = _swap_repair(rng, chk_sock, var_sock, rng.permutation(len(var_sock)), M, N)
    vs = var_sock[perm]
    order = np.lexsort((vs, chk_sock))        # check-major, variables ascending
    chk, vs = chk_sock[order], vs[order]
    row_ptr = np.zeros(M + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(np.bincount(chk, minlength=M))
    lrng = np.random.default_rng(seed_labels)
    val = lrng.integers(1, 1 << m, size=len(vs)).astype(np.uint16)
    return Code(M, N, m, row_ptr, vs.astype(np.int32), val,
                default_poly(m) if poly is None else poly,
                {"graph": seed_graph, "labels": seed_labels})


def _has_double(chk, var, M, N) -> bool:
    key = chk.astype(np.int64) * N + var
    return len(np.unique(key)) != len(key)


def _swap_repair(rng, chk, var_sock, perm, M, N):
    perm = perm.copy()
    for _ in range(100000):
        key = chk.astype(np.int64) * N + var_sock[perm]
        uniq, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
        dup = np.nonzero(cnt[inv] > 1)[0]
        if len(dup) == 0:
            return perm
        a = dup[0]
        b = rng.integers(len(perm))
        perm[a], perm[b] = perm[b], perm[a]
    raise RuntimeError("could not remove double edges")


def make_tree_code(n_checks: int, m: int, seed: int, poly: int | None = None) -> Code:
    """A random cycle-free Tanner graph (necessarily irregular): each new check
    attaches to one existing variable and brings 1-2 new variables."""
    rng = np.random.default_rng(seed)
    edges = []                     # (check, var)
    nvar = rng.integers(2, 4)
    edges += [(0, v) for v in range(nvar)]
    for c in range(1, n_checks):
        anchor = int(rng.integers(nvar))
        newv = int(rng.integers(1, 3))
        edges.append((c, anchor))
        for t in range(newv):
            edges.append((c, nvar + t))
        nvar += newv
    edges.sort()
    chk = np.array([e[0] for e in edges])
    var = np.array([e[1] for e in edges])
    row_ptr = np.zeros(n_checks + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(np.bincount(chk, minlength=n_checks))
    val = rng.integers(1, 1 << m, size=len(var)).astype(np.uint16)
    return Code(n_checks, nvar, m, row_ptr, var.astype(np.int32), val,
                default_poly(m) if poly is None else poly, {"tree": seed})


class Encoder:
    """Systematic encoder from Gaussian elimination of H over GF(2^m)."""

    def __init__(self, code: Code):
        self.code = code
        f = self.f = _Field(code.m, code.poly)
        H = code.dense()
        M, N = H.shape
        R = H.copy()
        pivots = []
        row = 0
        for col in range(N):
            if row == M:
                break
            nz = np.nonzero(R[row:, col])[0]
            if len(nz) == 0:
                continue
            r = row + nz[0]
            R[[row, r]] = R[[r, row]]
            R[row] = f.mul(f.inv(R[row, col]), R[row])
            for rr in range(M):
                if rr != row and R[rr, col] != 0:
                    R[rr] ^= f.mul(R[rr, col], R[row])
            pivots.append(col)
            row += 1
        self.rank = len(pivots)
        self.pivots = np.array(pivots, dtype=np.int64)
        self.info_pos = np.array([c for c in range(N) if c not in set(pivots)], dtype=np.int64)
        self.R = R[: self.rank]
        self.K = len(self.info_pos)

    def encode(self, info: np.ndarray) -> np.ndarray:
        """info [F, K] symbols -> codewords [F, N]."""
        info = np.asarray(info, dtype=np.int64)
        F = info.shape[0]
        cw = np.zeros((F, self.code.N), dtype=np.int64)
        cw[:, self.info_pos] = info
        # in RREF: x_p + sum_{j not pivot} R[r, j] x_j = 0 -> x_p = sum R[r, j] x_j
        for r, p in enumerate(self.pivots):
            acc = np.zeros(F, dtype=np.int64)
            for jcol in self.info_pos:
                a = self.R[r, jcol]
                if a:
                    acc ^= self.f.mul(a, cw[:, jcol])
            cw[:, p] = acc
        return cw

    def syndrome(self, cw: np.ndarray) -> np.ndarray:
        """H x for words [F, N] (integer check used by tests and benchmarks)."""
        c = self.code
        s = np.zeros((cw.shape[0], c.M), dtype=np.int64)
        for ch in range(c.M):
            for e in range(c.row_ptr[ch], c.row_ptr[ch + 1]):
                s[:, ch] ^= self.f.mul(int(c.val[e]), cw[:, c.col[e]])
        return s


def random_codewords(enc: Encoder, F: int, seed: int = 1003) -> np.ndarray:
    rng = np.random.default_rng(seed)
    info = rng.integers(0, enc.code.q, size=(F, enc.K))
    return enc.encode(info)


def sigma2_from_ebn0(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def bpsk_awgn_llr(cw: np.ndarray, m: int, ebn0_db: float, rate: float, seed: int = 1004,
                  dtype=np.float32) -> np.ndarray:
    """Channel LLRs [F, N, m] for codewords [F, N] over BPSK/AWGN."""
    s2 = sigma2_from_ebn0(ebn0_db, rate)
    bits = (cw[..., None] >> np.arange(m)) & 1
    x = 1.0 - 2.0 * bits
    rng = np.random.default_rng(seed)
    y = x + np.sqrt(s2) * rng.standard_normal(x.shape)
    return (2.0 * y / s2).astype(dtype)


# --- workloads --------------------------------------------------------------
# Parity/benchmark configurations: (name, m, k, N, frames, EbN0 list, max_iter)
WORKLOADS = {
    "gf4_n96": dict(m=2, k=4, N=96, frames=1000, ebn0=[2.0], max_iter=50),
    "gf64_n1000": dict(m=6, k=6, N=1000, frames=4096, ebn0=[2.0, 2.25, 2.5, 2.75, 3.0], max_iter=100),
    "gf256_n512": dict(m=8, k=8, N=512, frames=8192, ebn0=[3.0], max_iter=100),
    "gf16_n2048": dict(m=4, k=4, N=2048, frames=3000, ebn0=[2.5], max_iter=100),
    "gf64_n512": dict(m=6, k=6, N=512, frames=6000, ebn0=[2.5], max_iter=100),
    "gf256_n256_k16": dict(m=8, k=16, N=256, frames=2000, ebn0=[2.5], max_iter=100),
    # irregular column weights (Sec. 2 notes the extension): 70% weight 2,
    # 20% weight 3, 10% weight 4; near-regular rows of weight ~6
    "gf64_n1000_irr": dict(m=6, k=6, N=1000, frames=2048, ebn0=[2.0, 2.5, 3.0], max_iter=100,
                           var_dist={2: 0.7, 3: 0.2, 4: 0.1}),
}


@dataclass
class Batch:
    code: Code
    enc: Encoder
    cw: np.ndarray
    llr: np.ndarray
    ebn0: float
    sigma2: float

    @property
    def info_bits_per_frame(self) -> int:
        return self.enc.K * self.code.m


def make_batch(name: str, frames: int | None = None, ebn0: float | None = None,
               point: int = 0, seed_base: int = 1000) -> Batch:
    w = WORKLOADS[name]
    vd = irregular_var_degrees(w["N"], w["var_dist"], seed=seed_base + 5) if "var_dist" in w else None
    code = make_code(w["N"], w["k"], w["m"], seed_graph=seed_base + 1, seed_labels=seed_base + 2, var_degrees=vd)
    enc = Encoder(code)
    F = w["frames"] if frames is None else frames
    e = w["ebn0"][point] if ebn0 is None else ebn0
    cw = random_codewords(enc, F, seed=seed_base + 3 + 10 * point)
    llr = bpsk_awgn_llr(cw, code.m, e, code.design_rate, seed=seed_base + 4 + 10 * point)
    return Batch(code, enc, cw, llr, e, sigma2_from_ebn0(e, code.design_rate))
