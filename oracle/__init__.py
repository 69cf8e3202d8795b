"""CPU FP64 oracle for the LOCC crop-collision path.  TEST INFRASTRUCTURE ONLY.

Imported by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark, never by the product path.  See ``locc_oracle`` for what it computes.
"""
from . import locc_oracle  # noqa: F401
