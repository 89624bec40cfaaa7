"""CPU FP64 oracle for the Cahn-Hilliard spectral stepper, its adjoint and the conv surrogate.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product path (the HIP library and its Python binding).
"""
from . import ch, adjoint  # noqa: F401
