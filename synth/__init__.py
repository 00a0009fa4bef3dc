"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *draws* inputs: prescribed spectra, random unitary bases,
Hermitian test matrices with a known spectrum, random start blocks and loss
weights.  It holds none of the eigensolver's arithmetic, so both the CPU
oracle and the GPU library can be fed from it without sharing any code.
"""
from .problems import (  # noqa: F401
    Problem,
    complex_gaussian,
    dft_like_spectrum,
    gaussian_unitary,
    hermitian_from_spectrum,
    make_problem,
    real_gaussian,
    symmetric_from_spectrum,
    uniform_spectrum,
    CFG_PARITY,
)
