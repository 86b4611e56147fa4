"""Conversions between oracle messages (probability domain) and the decoder's
state format (signed log2 magnitude of the Fourier image), plus tolerances."""
import numpy as np

from oracle.gf import hadamard

LMAX = 100.0
# Norm-wise tolerance on linear Fourier-domain messages (|P| <= 1) for FP32.
TOL_FP32 = 1e-4
# Bits whose Fourier-domain posterior value is within TAU of zero (relative to
# Q(0) = 1) may legitimately flip between FP32 and FP64.
TAU = 1e-5


def to_state(p: np.ndarray) -> np.ndarray:
    """Prob-domain messages [F, E, q] -> signed log2 words of P = WHT(p)."""
    q = p.shape[-1]
    P = p @ hadamard(q).T
    with np.errstate(divide="ignore"):
        # + 0.0 turns the -0.0 that -log2(1.0) yields into +0.0: a set sign bit
        # with magnitude 0 would encode P = -1
        mag = np.clip(-np.log2(np.abs(P)), 0.0, LMAX) + 0.0
    return np.where(P < 0, -mag, mag).astype(np.float32)


def from_state(w: np.ndarray) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    return np.where(np.signbit(w), -1.0, 1.0) * np.exp2(-np.abs(w))


def fourier(p: np.ndarray) -> np.ndarray:
    return p @ hadamard(p.shape[-1]).T


def near_tie_bits(qbits: np.ndarray) -> np.ndarray:
    """[F, N] mask of symbols with a hard-decision bit near a tie."""
    return (np.abs(qbits) < TAU).any(-1)


def fsynd_near_tie(tc, post: np.ndarray) -> np.ndarray:
    """[F, M] mask of checks whose Fourier syndrome involves a near-zero value."""
    Q = fourier(post)
    F = post.shape[0]
    mask = np.zeros((F, tc.M), dtype=bool)
    for e in range(tc.E):
        vals = Q[:, tc.edge_var[e], tc.fsyn_pts[e]]
        mask[:, tc.edge_check[e]] |= (np.abs(vals) < TAU).any(-1)
    return mask


def store_pmf(qp: np.ndarray, prec: str) -> np.ndarray:
    """Messages as 16-bit storage holds them: qp = q times a message's pmf (for
    instance the inverse transform of its Fourier image), clamped at zero,
    rounded to FP32 and then to FP16 (nearest even) or BF16 (nearest even on
    the FP32 word).  Returns the stored values widened to FP64 (still times q)."""
    v = np.maximum(np.asarray(qp, dtype=np.float64), 0.0).astype(np.float32)
    if prec == "fp16":
        return v.astype(np.float16).astype(np.float64)
    if prec == "bf16":
        u = v.view(np.uint32).astype(np.uint64)
        r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
        return r.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(prec)
