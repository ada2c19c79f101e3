"""Input generator checks: the SIPG operators are the ones Section 4 describes.

Pins: manufactured-solution L2 rates p+1 (textbook SIPG behaviour),
symmetry, positive definiteness of the Poisson operator, convergence of the
impedance Helmholtz discretisation, and the partition's geometry.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workloads import configs, partition, sipg


def _exact(x, y):
    return np.sin(np.pi * x) * np.sin(np.pi * y)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_poisson_l2_rate(p):
    errs = []
    for n in (4, 8):
        A = sipg.assemble(n, p)
        b = sipg.load_vector(n, p, lambda x, y: 2 * np.pi ** 2 * _exact(x, y))
        u = spla.spsolve(A.to_scipy().tocsc(), b)
        errs.append(sipg.l2_error(n, p, u, _exact))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p + 1 - 0.25


def test_symmetry_and_spd():
    A = sipg.assemble(4, 2)
    D = A.to_dense()
    assert np.array_equal(D, D.T)
    np.linalg.cholesky(D)          # Poisson SIPG with penalty 10 p^2/h is SPD
    H = sipg.assemble(4, 2, "helmholtz", kappa=12.0).to_dense()
    assert np.array_equal(H, H.T)  # complex symmetric, not Hermitian
    assert np.abs(H - H.conj().T).max() > 0


def test_varcoef_symmetric_spd():
    rng = np.random.default_rng(0)
    coef = np.exp(configs.grf(6, 0.1, 1.0, rng))
    D = sipg.assemble(6, 1, coef=coef).to_dense()
    assert np.allclose(D, D.T, rtol=0, atol=1e-12 * np.abs(D).max())
    np.linalg.cholesky(D)


def _impedance_load(n, p, kappa):
    """rhs for u = sin(pi x) sin(pi y): f = (2 pi^2 - kappa^2) u and the
    impedance data g = du/dn - i kappa u = -pi sin(pi s) on every side."""
    b = sipg.load_vector(n, p, lambda x, y: (2 * np.pi ** 2 - kappa ** 2) * _exact(x, y)).astype(complex)
    L = sipg.Lagrange1D(p)
    xq, wq = sipg.gauss_rule(p + 3)
    Bq = L.value(xq)
    q = (p + 1) ** 2
    h = 1.0 / n
    e0, e1 = L.value(0.0)[0], L.value(1.0)[0]
    for k in range(n):
        s = (k + xq) * h
        g = -np.pi * np.sin(np.pi * s)
        tang = Bq.T @ (wq * g * h)                  # along the side
        for (ex, ey, ev, axis) in ((0, k, e0, "x"), (n - 1, k, e1, "x"),
                                   (k, 0, e0, "y"), (k, n - 1, e1, "y")):
            e = ex + n * ey
            loc = np.outer(tang, ev) if axis == "x" else np.outer(ev, tang)
            b[e * q:(e + 1) * q] += loc.reshape(-1)
    return b


def test_helmholtz_impedance_converges():
    kappa = 6.0
    p = 2
    errs = []
    for n in (4, 8):
        A = sipg.assemble(n, p, "helmholtz", kappa=kappa)
        b = _impedance_load(n, p, kappa)
        u = spla.spsolve(A.to_scipy().tocsc(), b)
        errs.append(sipg.l2_error(n, p, u, _exact))
    assert np.log2(errs[0] / errs[1]) > p + 1 - 0.3


def test_point_source_partition_of_unity():
    b = sipg.point_source(8, 3, 0.3712, 0.8123)
    assert abs(b.sum() - 1.0) < 1e-12        # Lagrange basis sums to one
    assert np.count_nonzero(b) <= 16


def test_partition_geometry():
    t = partition.build_tree(16, 16, 16)
    assert t.n_leaves == 16
    assert sorted(t.leaf_elems.tolist()) == list(range(256))
    assert t.boxes[2].y1 == 8 and t.boxes[2].x1 == 16     # first cut splits y
    t2 = partition.build_tree(37, 37, 16)                 # uneven grids
    assert sorted(t2.leaf_elems.tolist()) == list(range(37 * 37))
    assert all(b.w >= 2 and b.h >= 2 for b in t2.boxes.values())
    sizes = np.diff(t2.leaf_ptr)
    assert sizes.max() <= 16
