"""Seeded synthetic inputs (DG operators, box trees, right-hand sides).

Shared by the oracle and the library's tests and benchmark; holds no part of
the preconditioner's arithmetic.
"""
from . import configs, partition, sipg  # noqa: F401
