"""CPU oracle for MG-preconditioned CG on the 27-point stencil.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU library never does.
"""
from .pyoracle import Oracle  # noqa: F401
