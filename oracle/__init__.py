"""FP64 CPU oracle of the two-body macro-ion PIC step.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product path.
"""
from .oracle import Oracle, ORACLE_LIB, split_momentum, ac_from_omega  # noqa: F401
