"""MI355X implementation of the low-rank Schur-complement (HSS) nested-dissection
preconditioner: a C-ABI library (include/hss.h, csrc/) and its ctypes binding."""
