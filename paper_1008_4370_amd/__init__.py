"""MI355X (gfx950) decoder for (2,k) non-binary LDPC codes over GF(2^m) using the
Log-Fourier sum-product algorithm of Kasai & Sakaniwa (arXiv:1008.4370).

The decoding path is the C-ABI library ``libldpcfd.so`` (hand-written HIP
kernels); ``paper_1008_4370_amd.decoder`` is a thin ctypes binding over it.
Importing this package does not load the library; ``decoder`` does, and fails
loudly when it is missing.
"""
__all__ = ["synth", "decoder"]
