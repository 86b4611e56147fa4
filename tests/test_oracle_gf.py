"""Pins of the oracle's field arithmetic, transforms and signed-log map."""
import os

import numpy as np
import pytest

from oracle.gf import DEFAULT_POLY, GF, dot, hadamard
from oracle.lfsp import gamma, gamma_inv
from oracle.sp import channel_prior, fourier, xor_conv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_gf8_table_matches_paper():
    """Sec. 2: the m-bit representation of GF(8) with alpha^3 + alpha + 1 = 0."""
    g = GF(3, 0b1011)
    for row in _read("gf8_table.txt"):
        bits = [int(b) for b in row[1:]]
        x = 0 if row[0] == "zero" else g.alpha_pow(int(row[0]))
        assert list(g.bits(x)) == bits, row


def test_dot_product_example():
    """Sec. 2.1 example: z.x = 3 for the printed 8-bit vectors."""
    rows = {r[0]: r[1:] for r in _read("dot_example.txt")}
    z = sum(int(b) << i for i, b in enumerate(rows["z"]))
    x = sum(int(b) << i for i, b in enumerate(rows["x"]))
    assert dot(z, x) == int(rows["dot"][0])
    H = hadamard(256)
    assert H[z, x] == (-1) ** int(rows["dot"][0])


@pytest.mark.parametrize("m", range(1, 9))
def test_default_polys_primitive(m):
    g = GF(m)
    a = g.alpha_pow(1)
    assert g.order(a) == (1 << m) - 1


@pytest.mark.parametrize("m", range(1, 9))
def test_companion_matrix_is_multiplication_by_alpha(m):
    """Appendix A: A^i alpha^j = alpha^(i+j) with A the printed companion matrix."""
    g = GF(m)
    A = g.companion()
    assert np.array_equal(A % 2, g.mat(g.alpha_pow(1)))
    Ai = np.eye(m, dtype=np.int64)
    for i in range(min(g.q - 1, 20)):
        for j in range(min(g.q - 1, 20)):
            assert g.apply(Ai, g.alpha_pow(j)) == g.alpha_pow(i + j)
        Ai = (A @ Ai) % 2


@pytest.mark.parametrize("m", [2, 3, 5, 8])
def test_field_axioms_and_matrix_homomorphism(m):
    g = GF(m)
    rng = np.random.default_rng(m)
    for _ in range(200):
        a, b, c = (int(v) for v in rng.integers(0, g.q, 3))
        assert g.mul(g.mul(a, b), c) == g.mul(a, g.mul(b, c))
        assert g.mul(a, b ^ c) == g.mul(a, b) ^ g.mul(a, c)
        assert np.array_equal((g.mat(a) @ g.mat(b)) % 2, g.mat(int(g.mul(a, b))))
        if a:
            assert g.mul(a, g.inv(a)) == 1


@pytest.mark.parametrize("m", range(1, 9))
def test_hadamard_squares_to_q_identity(m):
    q = 1 << m
    H = hadamard(q)
    assert np.array_equal(H @ H, q * np.eye(q))


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6])
def test_convolution_theorem(m):
    """Sec. 2.1: the Fourier transform turns XOR convolution into products."""
    q = 1 << m
    rng = np.random.default_rng(10 + m)
    H = hadamard(q)
    xt = np.arange(q)[:, None] ^ np.arange(q)[None, :]
    p1, p2 = rng.random((2, 5, q))
    lhs = fourier(xor_conv(p1, p2, xt), H)
    rhs = fourier(p1, H) * fourier(p2, H)
    assert np.allclose(lhs, rhs, atol=1e-12)
    # brute force of the convolution itself on one vector
    bf = np.array([sum(p1[0, a] * p2[0, b] for a in range(q) for b in range(q) if a ^ b == x)
                   for x in range(q)])
    assert np.allclose(xor_conv(p1, p2, xt)[0], bf)


@pytest.mark.parametrize("m", [3, 4, 5, 6])
def test_fourier_label_map_direction(m):
    """Appendix A (reading: H_cv = M_h^T): the transform of p(h^-1 x) is P(M_h^T z)
    for every label h; the untransposed map M_h z fails for some h."""
    g = GF(m)
    q = g.q
    H = hadamard(q)
    rng = np.random.default_rng(m)
    p = rng.random(q)
    P = fourier(p, H)
    xs = np.arange(q)
    untransposed_fails = False
    for h in range(1, q):
        pt = p[g.mul(g.inv(h), xs)]
        Pt = fourier(pt, H)
        assert np.allclose(Pt, P[g.fourier_perm(h)], atol=1e-12), h
        Mz = np.array([g.apply(g.mat(h), z) for z in range(q)])
        if not np.allclose(Pt, P[Mz], atol=1e-9):
            untransposed_fails = True
    assert untransposed_fails


def test_gamma_is_a_homomorphism():
    """Sec. 3.2: Gamma(xy) = Gamma(x) + Gamma(y) (sign XOR, log add)."""
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 1000)
    y = rng.uniform(-1, 1, 1000)
    sx, lx = gamma(x)
    sy, ly = gamma(y)
    sxy, lxy = gamma(x * y)
    assert np.array_equal(sxy, sx ^ sy)
    assert np.allclose(lxy, lx + ly)
    assert np.allclose(gamma_inv(*gamma(x)), x)
    assert gamma(np.array([0.0]))[0][0] == 0      # sgn(0) fixed to 0


@pytest.mark.parametrize("m", [1, 2, 4, 6])
def test_channel_prior_closed_form(m):
    """Fourier transform of the BPSK symbol pmf: P(z) = prod_{i in z} tanh(L_i/2)
    (the Gallager-f view of the Log-Fourier initial message, Sec. 5)."""
    q = 1 << m
    rng = np.random.default_rng(m)
    L = rng.normal(0, 4, (7, m))
    p0 = channel_prior(L, m)
    assert np.allclose(p0.sum(-1), 1.0)
    P0 = fourier(p0, hadamard(q))
    t = np.tanh(L / 2)
    for z in range(q):
        expect = np.prod([t[:, i] for i in range(m) if (z >> i) & 1], axis=0) if z else np.ones(7)
        assert np.allclose(P0[:, z], expect, atol=1e-12)
    # bit marginals of the pmf are the per-bit posteriors sigma(L)
    xs = np.arange(q)
    for i in range(m):
        assert np.allclose(p0[:, ((xs >> i) & 1) == 0].sum(-1), 1 / (1 + np.exp(-L[:, i])))
