"""CPU oracle: a plain FP64 / complex128 implementation of the preconditioner.

Test infrastructure only. The tests, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the library; the library never
imports, links or runs anything from here, and this package imports nothing
from the library.
"""
