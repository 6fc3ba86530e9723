"""CPU FP64 oracle for the streaming GCP hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the product package, and sharing no code
with it.  Each module cites the part of the paper it follows.
"""
from . import gcp, solve, adam, window  # noqa: F401
