"""GF(2^m) arithmetic for the oracle (test infrastructure only).

Representation (Sec. 2, the GF(8) example with alpha^3 + alpha + 1 = 0): a
symbol x is the m-bit vector (x_1, ..., x_m) of its coefficients in the basis
1, alpha, ..., alpha^(m-1); as an integer, x_i is bit (i-1).  Multiplication
is polynomial multiplication reduced modulo the primitive polynomial pi(x).

Label maps (Appendix A): multiplication by a fixed h is GF(2)-linear on the
bit vectors; ``mat(h)`` is its m x m matrix M_h (acting on column vectors),
``companion()`` is the paper's companion matrix A of pi(x), and for h = alpha^i
M_h = A^i.  The Fourier-domain label map of the check-to-variable step is
z -> M_h^T z (the paper's H_cv z with H_cv = (A^i)^T); see ``fourier_perm``.

The primitive polynomials for m != 3 are not given in the paper; the defaults
below are standard primitive trinomials/pentanomials (each checked to have
alpha of order 2^m - 1 by the oracle tests).
"""
from __future__ import annotations

import numpy as np

# pi(x) as an integer: bit j = coefficient of x^j (bit m set).
DEFAULT_POLY = {
    1: 0b11,          # x + 1
    2: 0b111,         # x^2 + x + 1
    3: 0b1011,        # x^3 + x + 1        (the paper's GF(8) example, Sec. 2)
    4: 0b10011,       # x^4 + x + 1
    5: 0b100101,      # x^5 + x^2 + 1
    6: 0b1000011,     # x^6 + x + 1
    7: 0b10001001,    # x^7 + x^3 + 1
    8: 0b100011101,   # x^8 + x^4 + x^3 + x^2 + 1
}


class GF:
    """GF(2^m) with a fixed primitive element alpha (the class of x)."""

    def __init__(self, m: int, poly: int | None = None):
        if not 1 <= m <= 8:
            raise ValueError("m must be in 1..8")
        self.m = m
        self.q = 1 << m
        self.poly = DEFAULT_POLY[m] if poly is None else int(poly)
        if self.poly >> m != 1:
            raise ValueError("poly must have degree m")
        q = self.q
        # full multiplication table by the definition (shift-and-add mod pi)
        self.mul_table = np.zeros((q, q), dtype=np.int64)
        for a in range(q):
            for b in range(q):
                self.mul_table[a, b] = self._mul_def(a, b)
        self.inv_table = np.zeros(q, dtype=np.int64)
        for a in range(1, q):
            hits = np.nonzero(self.mul_table[a] == 1)[0]
            if len(hits) != 1:
                raise ValueError("polynomial is not irreducible")
            self.inv_table[a] = hits[0]

    # -- scalar arithmetic -------------------------------------------------
    def _mul_def(self, a: int, b: int) -> int:
        """Polynomial product of a and b reduced modulo pi(x)."""
        r = 0
        while b:
            if b & 1:
                r ^= a
            b >>= 1
            a <<= 1
            if (a >> self.m) & 1:
                a ^= self.poly
        return r

    def mul(self, a, b):
        return self.mul_table[a, b]

    def inv(self, a):
        a = np.asarray(a)
        if np.any(a == 0):
            raise ZeroDivisionError("0 has no inverse")
        return self.inv_table[a]

    def alpha_pow(self, i: int) -> int:
        """alpha^i for a primitive alpha (the element x, integer 2; for m=1, 1)."""
        a = 2 if self.m > 1 else 1
        r = 1
        for _ in range(i % (self.q - 1) if self.q > 2 else 0):
            r = self._mul_def(r, a)
        return r

    def order(self, a: int) -> int:
        """Multiplicative order of a nonzero element."""
        r, n = a, 1
        while r != 1:
            r = self._mul_def(r, a)
            n += 1
        return n

    # -- bit vectors and matrices (Appendix A) ---------------------------
    def bits(self, x: int) -> np.ndarray:
        """m-bit column vector (x_1..x_m), x_i = bit (i-1) of x."""
        return np.array([(x >> i) & 1 for i in range(self.m)], dtype=np.int64)

    def from_bits(self, v) -> int:
        v = np.asarray(v) % 2
        return int(sum(int(v[i]) << i for i in range(self.m)))

    def mat(self, h: int) -> np.ndarray:
        """M_h: GF(2) matrix with M_h @ bits(x) = bits(h*x) (mod 2)."""
        cols = [self.bits(self._mul_def(h, 1 << j)) for j in range(self.m)]
        return np.stack(cols, axis=1)

    def companion(self) -> np.ndarray:
        """Companion matrix A of pi(x) exactly as printed in Appendix A:
        ones on the sub-diagonal, (pi_0, ..., pi_{m-1}) in the last column."""
        m = self.m
        A = np.zeros((m, m), dtype=np.int64)
        for i in range(1, m):
            A[i, i - 1] = 1
        for i in range(m):
            A[i, m - 1] = (self.poly >> i) & 1
        return A

    def apply(self, Mat: np.ndarray, x: int) -> int:
        """Integer of Mat @ bits(x) over GF(2)."""
        return self.from_bits(Mat @ self.bits(x))

    def fourier_perm(self, h: int) -> np.ndarray:
        """perm[z] = integer of M_h^T z.

        The Fourier transform of p~(x) = p(h^-1 x) is P~(z) = P(M_h^T z)
        (Appendix A, with the reading H_cv = M_h^T = (A^i)^T)."""
        MT = self.mat(h).T
        return np.array([self.apply(MT, z) for z in range(self.q)], dtype=np.int64)


def popcount_parity(a: np.ndarray) -> np.ndarray:
    """Parity of the number of set bits of each integer in a (values < 2^16)."""
    a = np.asarray(a, dtype=np.int64)
    p = np.zeros_like(a)
    for i in range(16):
        p ^= (a >> i) & 1
    return p


def hadamard(q: int) -> np.ndarray:
    """Sylvester-Hadamard matrix H[z, x] = (-1)^(z . x), z . x = sum_i z_i x_i
    (the Fourier transform of Sec. 2.1)."""
    idx = np.arange(q)
    return (1 - 2 * popcount_parity(idx[:, None] & idx[None, :])).astype(np.float64)


def dot(z: int, x: int) -> int:
    """z . x = sum_i z_i x_i over the integers (Sec. 2.1 example)."""
    return bin(int(z) & int(x)).count("1")
