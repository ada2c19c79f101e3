"""The Section 4 study families of the workload generator (host only): real
symmetric operators with the coefficients the paper's problems prescribe."""
import math

import numpy as np

from workloads import configs


def test_study_operators():
    n, p = 8, 2
    base = configs.study("poisson", n, p).op.to_dense()
    for kind in ("poisson", "cavity", "aniso", "contrast"):
        P = configs.study(kind, n, p)
        A = P.op.to_dense()
        assert not P.op.is_complex and np.abs(A - A.T).max() == 0.0
        assert P.prec == "fp64" and P.tol == configs.STUDY_TOL[kind]
    # the soft cavity differs from Poisson by -kappa^2 times the (block-diagonal,
    # positive definite) mass matrix, with kappa at 8 DG nodes per wavelength
    cav = configs.study("cavity", n, p)
    assert math.isclose(cav.kappa, 2 * math.pi * n * (p + 1) / 8.0)
    D = (cav.op.to_dense() - base) / (-cav.kappa ** 2)
    q = (p + 1) ** 2
    for e in range(n * n):
        blk = D[e * q:(e + 1) * q, e * q:(e + 1) * q]
        assert np.linalg.eigvalsh(blk).min() > 0
        D[e * q:(e + 1) * q, e * q:(e + 1) * q] = 0
    assert np.abs(D).max() < 1e-12
    # equation (60) normalized, with a0 = 1: c0 adds c0 times that mass matrix
    a1 = configs.study("aniso", n, p, c0=2.0, a0=1.0).op.to_dense()
    assert np.abs((a1 - base) / 2.0 + (cav.op.to_dense() - base) / cav.kappa ** 2).max() < 1e-9


def test_contrast_enclosure():
    n = 16
    c = configs.contrast_coef(n, 1e3)
    xc = (np.arange(n) + 0.5) / n
    for ey in range(n):
        for ex in range(n):
            inside = 0.125 < xc[ex] < 0.875 and 0.375 < xc[ey] < 0.5
            assert c[ey, ex] == (1e-3 if inside else 1.0)
    assert (c < 1).sum() == 12 * 2  # 12 columns (x) by 2 rows (y) of elements
