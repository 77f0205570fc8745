"""CPU FP64 oracle for SRP-PHAT mapping and its Nyquist-Shannon approximation.

TEST INFRASTRUCTURE ONLY. This package is the checker the GPU library is
compared against. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or call it; the product path never
does, and it shares no code, tables or constants with the HIP library.

Everything is plain NumPy in float64, written from Dietzen, De Sena and van
Waterschoot, "Low-Complexity Steered Response Power Mapping based on
Nyquist-Shannon Sampling" (WASPAA 2021). Each function names the section and
equation it follows. Library primitives used as steps: numpy.fft.rfft, complex
exponentials, numpy.sinc and matrix products (BLAS).

Parity status: every function is pinned by a CPU test against the paper's
printed numbers, a closed form, an identity between two of the paper's forms
or brute force on tiny inputs; see tests/test_oracle.py.
"""
from .srp_oracle import *  # noqa: F401,F403
