"""Philox4x32-10 counter-based generator and the Gaussian test matrices.

Philox4x32-10 is taken from its published definition (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a
4 x 32-bit counter, a 2 x 32-bit key, ten rounds of two 32x32->64
multiplies with the Weyl key schedule in between.

The randomized HSS construction of Theorem 1 (Section 1) draws Gaussian
test vectors; the oracle and the library each generate them from this
same definition so that both see the same test matrices. Entry (r, c) of
the test matrix of tree node ``node`` uses counter (r, c, node, stream)
and key (seed mod 2^32, seed div 2^32); Box-Muller turns the first two
output words into a standard normal (real case) or into
(g1 + i g2)/sqrt(2) (complex case).

Test infrastructure only: nothing in the library imports this module.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint32 counter arrays; returns 4 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.asarray(c1, dtype=np.uint64) & MASK
    c2 = np.asarray(c2, dtype=np.uint64) & MASK
    c3 = np.asarray(c3, dtype=np.uint64) & MASK
    k0 = np.uint64(k0) & MASK
    k1 = np.uint64(k1) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return c0, c1, c2, c3


def gaussian_matrix(seed: int, node: int, nrows: int, ncols: int, complex_: bool,
                    stream: int = 0) -> np.ndarray:
    """Test matrix Omega[r, c] for r < nrows, c < ncols of one tree node."""
    r = np.repeat(np.arange(nrows, dtype=np.uint64), ncols)
    c = np.tile(np.arange(ncols, dtype=np.uint64), nrows)
    x0, x1, _, _ = philox4x32_10(r, c, np.full_like(r, node), np.full_like(r, stream),
                                 int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    u1 = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (x1.astype(np.float64) + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    g1 = rad * np.cos(2.0 * np.pi * u2)
    if not complex_:
        return g1.reshape(nrows, ncols)
    g2 = rad * np.sin(2.0 * np.pi * u2)
    return ((g1 + 1j * g2) / np.sqrt(2.0)).reshape(nrows, ncols)
