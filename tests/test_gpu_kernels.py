"""Kernel-level GPU checks through the C ABI (hss_debug.h): the batched MFMA
GEMM and the batched Gauss-Jordan elimination against NumPy on ragged,
multi-tile shapes for every scalar type."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1508_07798_amd import hss  # noqa: E402

DT = {"float32": (np.float32, torch.float32, 2e-5), "float64": (np.float64, torch.float64, 1e-13),
      "complex64": (np.complex64, torch.complex64, 2e-5), "complex128": (np.complex128, torch.complex128, 1e-13)}


def _rand(rng, shape, npdt):
    a = rng.standard_normal(shape)
    if np.issubdtype(npdt, np.complexfloating):
        a = a + 1j * rng.standard_normal(shape)
    return a.astype(npdt)


def _dev(a, tdt):
    # column-major matrix a (rows x cols) as a CUDA tensor holding a.T in row-major order
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda")


@pytest.mark.parametrize("name", list(DT))
def test_batched_gemm(name):
    npdt, tdt, tol = DT[name]
    rng = np.random.default_rng(7)
    shapes = [(70, 45, 33), (1, 130, 7), (64, 64, 64), (129, 3, 200), (200, 150, 1)]
    As, Bs, Cs, ref = [], [], [], []
    alpha, beta = (-1.0, 1.0)
    for (m, n, k) in shapes:
        A = _rand(rng, (m, k), npdt)
        B = _rand(rng, (k, n), npdt)
        Cm = _rand(rng, (m, n), npdt)
        ref.append(alpha * (A.astype(np.complex128) @ B.astype(np.complex128)) + beta * Cm)
        As.append(_dev(A, tdt))
        Bs.append(_dev(B, tdt))
        Cs.append(_dev(Cm, tdt))
    hss.debug_gemm(As, Bs, Cs, alpha=alpha, beta=beta)
    for (m, n, k), Cd, R in zip(shapes, Cs, ref):
        got = Cd.cpu().numpy().T
        scale = np.sqrt(k) * 10 + 1
        assert np.abs(got - R).max() <= tol * scale * max(1.0, np.abs(R).max()), (m, n, k)


def test_batched_gemm_bf16x3():
    """FP32 operands on BF16 matrix cores (hi / lo split, three products): about 16
    significant bits per product, i.e. far better than plain BF16 (~4e-3)."""
    print("bf16x3 gemm", flush=True)
    rng = np.random.default_rng(9)
    shapes = [(70, 45, 33), (1, 130, 7), (64, 64, 64), (129, 3, 200), (200, 150, 1), (300, 257, 513)]
    As, Bs, Cs, ref, mag = [], [], [], [], []
    for (m, n, k) in shapes:
        A = rng.standard_normal((m, k)).astype(np.float32)
        B = rng.standard_normal((k, n)).astype(np.float32)
        Cm = rng.standard_normal((m, n)).astype(np.float32)
        ref.append(-(A.astype(np.float64) @ B.astype(np.float64)) + Cm)
        mag.append(np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)) + np.abs(Cm))
        As.append(_dev(A, torch.float32))
        Bs.append(_dev(B, torch.float32))
        Cs.append(_dev(Cm, torch.float32))
    hss.debug_gemm(As, Bs, Cs, alpha=-1.0, beta=1.0, bf16x3=True)
    for (m, n, k), Cd, R, Mg in zip(shapes, Cs, ref, mag):
        got = Cd.cpu().numpy().T.astype(np.float64)
        # each product carries a relative error below 2^-15; bound by the sum of |terms|
        assert np.all(np.abs(got - R) <= 4e-5 * Mg + 1e-6), (m, n, k)


GJ_CASES = [(name, 0, ((1, 3), (7, 0), (33, 20), (100, 45), (200, 230))) for name in DT]
# second-level blocks: forced narrow blocks over ragged sizes, and the automatic
# choice for blocks above 512 rows (128-column blocks, ragged last block)
GJ_CASES += [(name, 32, ((1, 3), (7, 0), (33, 20), (100, 45), (200, 230))) for name in DT]
GJ_CASES += [("float64", 0, ((600, 70), (530, 0), (40, 9))), ("complex64", 0, ((600, 70), (530, 0), (40, 9))),
             ("float32", 100, ((450, 30), (129, 1))),
             # tall real panels (six and eight rows per thread, single-precision pivot search)
             ("float64", 0, ((2600, 10), (3900, 0))),
             # complex double at root sizes (single-precision search, 256 and 512 threads)
             ("complex128", 0, ((1152, 20), (900, 0))),
             ("float32", 0, ((2000, 5), (1030, 3)))]


@pytest.mark.parametrize("name,block,sizes", GJ_CASES)
def test_batched_gauss_jordan(name, block, sizes):
    npdt, tdt, tol = DT[name]
    print(f"gj {name} block={block} sizes={sizes}", flush=True)
    rng = np.random.default_rng(11)
    mats, refs = [], []
    for n, m in sizes:
        # random matrices (pivoting needed) shifted to keep them reasonably conditioned
        A = _rand(rng, (n, n), npdt) + np.sqrt(n) * np.eye(n, dtype=npdt)
        B = _rand(rng, (n, m), npdt)
        M = np.concatenate([A, B], axis=1)
        mats.append(_dev(M, tdt))
        A64 = A.astype(np.complex128)
        refs.append((np.linalg.inv(A64), np.linalg.solve(A64, B.astype(np.complex128)) if m else None,
                     np.linalg.cond(A64)))
    sing = hss.debug_gj(mats, [s[0] for s in sizes], [s[1] for s in sizes], block=block)
    assert sing == 0
    for (n, m), Md, (Ainv, X, cond) in zip(sizes, mats, refs):
        got = Md.cpu().numpy().T
        e1 = np.abs(got[:, :n] - Ainv).max() / np.abs(Ainv).max()
        assert e1 <= tol * cond * 50, (n, e1, cond)
        if m:
            e2 = np.abs(got[:, n:] - X).max() / np.abs(X).max()
            assert e2 <= tol * cond * 50, (n, e2, cond)


def test_gauss_jordan_needs_pivoting_and_flags_singular():
    # a permutation-like matrix: no elimination without row interchanges
    n = 40
    P = np.eye(n)[np.random.default_rng(3).permutation(n)]
    A = P * 2.0 + 1e-3 * np.random.default_rng(4).standard_normal((n, n))
    M = _dev(A, torch.float64)
    assert hss.debug_gj([M], [n], [0]) == 0
    assert np.allclose(M.cpu().numpy().T, np.linalg.inv(A), atol=1e-10)
    Z = _dev(np.zeros((5, 5)), torch.float64)
    assert hss.debug_gj([Z], [5], [0]) == 1


def test_gauss_jordan_near_ties_in_double():
    """Double-precision panels pick pivots on a single-precision copy: rows whose
    moduli agree to single precision (a relative gap of 1e-12) may be taken in either
    order, and the inverse is still exact to double-precision rounding."""
    rng = np.random.default_rng(21)
    n = 300
    base = rng.standard_normal((n, n))
    A = base.copy()
    # every column gets a near-tie: two rows whose entries differ by a factor 1 + 1e-12,
    # both larger than the rest of the column
    for j in range(n):
        r1, r2 = rng.choice(n, 2, replace=False)
        big = 10.0 + rng.random()
        A[r1, j] = big
        A[r2, j] = -big * (1.0 + 1e-12)
    A += np.sqrt(n) * np.eye(n)
    M = _dev(A, torch.float64)
    assert hss.debug_gj([M], [n], [0]) == 0
    Ainv = np.linalg.inv(A)
    err = np.abs(M.cpu().numpy().T - Ainv).max() / np.abs(Ainv).max()
    assert err <= 1e-13 * np.linalg.cond(A) * 50, err
