"""FP64 CPU oracle for Fourier-domain Log-SP decoding of non-binary LDPC codes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables
or helpers with the HIP decoder in ``paper_1008_4370_amd``.

Contents (each function cites the passage of Kasai & Sakaniwa, "Fourier Domain
Decoding Algorithm of Non-Binary LDPC codes for Parallel Implementation",
IEICE Trans. Fundamentals 93(11), 2010 — arXiv:1008.4370 — that it follows):

* ``gf``    – GF(2^m) in the m-bit polynomial basis (Sec. 2) and the
              companion-matrix label maps (Appendix A).
* ``sp``    – the conventional probability-domain sum-product decoder with
              direct O(q^2) XOR convolutions (Sec. 2.1, Eq. (1)), plus the
              bitwise-MAP decision and both syndromes of Sec. 3.1/3.2.
              This is the plain definition the Log-Fourier method reaches
              exactly (up to rounding); it is THE oracle for parity.
* ``lfsp``  – a second, literal FP64 implementation of the Log-Fourier SP
              algorithm of Sec. 3.2 (signed-log messages, direct signed
              log-sum-exp log-convolution, Eq. (6)).  It is checked against
              ``sp`` and pins the reformulation (label-map direction, Gamma map,
              Fourier-domain decisions).

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against something other than itself (the paper's
GF(8) table and dot-product example, closed forms, brute-force marginals on
cycle-free codes, textbook binary BP, exact invariants).  FER/BER values,
iteration counts and timings have no printed value in the paper: parity
unpinned for those (only GPU-vs-oracle consistency applies).
"""
