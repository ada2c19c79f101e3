"""Pins of the oracle against facts that do not come from the oracle itself.

  * Philox: the published known-answer vectors.
  * Sets: the boundary rule checked against the dense matrix's sparsity
    (brute force); the per-level sizes of the 16x16, p=1 problem.
  * Schur complements: with tol = 0 every node's complement equals the
    Schur complement of A restricted to the node's box onto B (quotient
    property of Schur complements), computed from the dense matrix.
  * LDM^t: with tol = 0 the inverse factorization applied to b equals
    A^{-1} b and GMRES converges in one iteration.
  * ID: ||Z - U Z(J,:)||_F equals ||R22||_F; exact reproduction of
    low-rank matrices; the error is never below the SVD tail. On Kahan's
    matrix, where column pivoting alone leaves interpolation coefficients
    far above 2, the swaps bring every |T_ij| to at most 2 (the bound
    Section 1 puts on P), T is the least-squares interpolation of the free
    columns by the skeleton columns (numpy.linalg.lstsq), and |det R11|
    grows by more than 2 per swap.
  * HSS: tol -> 0 reproduces S; skeleton entries are reproduced exactly;
    off-diagonal blocks have the recorded rank; the judge bound holds.
  * GMRES: with P = I it converges in at most N steps to the dense solve.
    Restarted GMRES(m): every cycle's iterate equals the minimiser of the
    residual over x_c + M^{-1} K_m(A M^{-1}, r_c), computed independently by
    numpy.linalg.lstsq on an explicit Krylov basis.
  * MLP: back-propagation matches central differences; the first Adam step
    has the closed form -lr * sign(g).
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gmres as og
from oracle import hss as ohss
from oracle import mlp as omlp
from oracle import philox
from oracle.factor import OracleFactor
from oracle.sets import TreeSets, depth_of, hss_postorder
from workloads import configs, partition, sipg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    n = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            out = philox.philox4x32_10(*v[:6])
            assert [int(o) for o in out] == v[6:]
            n += 1
    assert n == 3


def test_gaussian_moments():
    G = philox.gaussian_matrix(1508, 7, 400, 50, False)
    assert abs(G.mean()) < 0.02 and abs(G.var() - 1) < 0.03
    C = philox.gaussian_matrix(1508, 7, 400, 50, True)
    assert abs(np.mean(np.abs(C) ** 2) - 1) < 0.03
    # the first columns do not depend on how many columns are drawn
    assert np.array_equal(philox.gaussian_matrix(3, 2, 10, 4, True),
                          philox.gaussian_matrix(3, 2, 10, 8, True)[:, :4])


def _small(n=8, p=1, pde="poisson", kappa=0.0):
    op = sipg.assemble(n, p, pde, kappa=kappa)
    tree = partition.build_tree(n, n, 16)
    return op, tree


def test_boundary_sets_brute_force():
    op, tree = _small(12, 1)
    T = TreeSets(op.row_ptr, op.col_idx, op.q, tree)
    D = op.to_dense()
    nz = D != 0
    for s in T.nodes:
        dofs = np.concatenate([np.arange(e * op.q, (e + 1) * op.q) for e in T.elems[s]])
        inside = np.zeros(op.ndof, bool)
        inside[dofs] = True
        bdf = [d for d in dofs if np.any(nz[d] & ~inside)]
        assert sorted(bdf) == sorted(T.sets[s].bdof.tolist())
        if T.sets[s].is_leaf:
            assert sorted(set(dofs) - set(bdf)) == sorted(T.sets[s].idof.tolist())
        else:
            mu, nu = T.sets[2 * s], T.sets[2 * s + 1]
            union = set(mu.bdof.tolist()) | set(nu.bdof.tolist())
            assert set(T.sets[s].bdof.tolist()) <= union
            assert sorted(union - set(bdf)) == sorted(T.sets[s].idof.tolist())
    # every dof is eliminated exactly once (interiors + root)
    allI = np.concatenate([T.sets[s].idof for s in T.nodes] + [T.root_idof])
    assert sorted(allI.tolist()) == list(range(op.ndof))


def test_level_sizes_poisson16():
    op, tree = _small(16, 1)
    T = TreeSets(op.row_ptr, op.col_idx, op.q, tree)
    want = {4: (16, 36, 28, 48), 3: (16, 24, 44, 72), 2: (56, 56, 60, 60), 1: (56, 56, 64, 64)}
    for d, (imin, imax, bmin, bmax) in want.items():
        ni = [T.sets[s].idof.size for s in T.nodes if depth_of(s) == d]
        nb = [T.sets[s].bdof.size for s in T.nodes if depth_of(s) == d]
        assert (min(ni), max(ni), min(nb), max(nb)) == (imin, imax, bmin, bmax)
    assert T.root_idof.size == 128


def test_parent_interior_run_leads_and_hss_cover():
    op, tree = _small(16, 2)
    T = TreeSets(op.row_ptr, op.col_idx, op.q, tree)
    for s in T.nodes:
        ns = T.sets[s]
        if s // 2 == 1:
            continue
        par_b = T.bset[s // 2]
        flags = [e not in par_b for e in ns.bnd_elems]
        m = ns.n_parent_interior
        assert all(flags[:m]) and not any(flags[m:])
        leaves = [t for t in hss_postorder(ns.hss) if t.is_leaf]
        cov = np.concatenate([np.arange(t.lo, t.hi) for t in leaves])
        assert np.array_equal(cov, np.arange(ns.bdof.size))
        assert all(t.hi - t.lo <= 4 * op.q for t in leaves)


def _brute_schur(D, box_dofs, bdof):
    inner = np.setdiff1d(box_dofs, bdof)
    Abb = D[np.ix_(bdof, bdof)]
    if inner.size == 0:
        return Abb
    return Abb - D[np.ix_(bdof, inner)] @ np.linalg.solve(D[np.ix_(inner, inner)], D[np.ix_(inner, bdof)])


@pytest.mark.parametrize("pde,p", [("poisson", 1), ("helmholtz", 2)])
def test_exact_schur_hierarchy(pde, p):
    op, tree = _small(8, p, pde, kappa=9.0)
    F = OracleFactor(op, tree, tol=0.0)
    D = op.to_dense()
    for s, nf in F.nodes.items():
        box = np.concatenate([np.arange(e * op.q, (e + 1) * op.q) for e in F.sets.elems[s]])
        Sb = _brute_schur(D, box, nf.bdof)
        assert np.linalg.norm(nf.S - Sb) <= 1e-11 * np.linalg.norm(Sb)


@pytest.mark.parametrize("pde,p", [("poisson", 1), ("poisson", 2), ("helmholtz", 2)])
def test_exact_ldmt_inverse_and_one_iteration(pde, p):
    op, tree = _small(8, p, pde, kappa=9.0)
    F = OracleFactor(op, tree, tol=0.0)
    D = op.to_dense()
    rng = np.random.default_rng(1)
    b = rng.standard_normal(op.ndof) + (1j * rng.standard_normal(op.ndof) if op.is_complex else 0)
    x = F.apply(b)
    xr = np.linalg.solve(D, b)
    assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.norm(xr) * np.linalg.cond(D) ** 0.5
    res = og.gmres(F.matvec, F.apply, b, tol=1e-10)
    assert res.iters == 1 and res.true_relres <= 1e-10


def test_row_id_identity_and_low_rank():
    rng = np.random.default_rng(2)
    m, l, r = 40, 30, 8
    H = rng.standard_normal((m, r)) @ rng.standard_normal((r, 200))
    Om = rng.standard_normal((200, l))
    Z = H @ Om
    rid = ohss.row_id(Z, 1e-10 * np.linalg.norm(Z), l)
    assert rid.k == r and not rid.exhausted
    err = np.linalg.norm(H - rid.U @ H[rid.skel])
    assert err <= 1e-9 * np.linalg.norm(H)
    # ||Z - U Z(J,:)||_F == ||R22||_F exactly, and never below the SVD tail
    Z2 = rng.standard_normal((25, 20)) * np.logspace(0, -6, 20)[None, :]
    for thr in (1e-1, 1e-3, 1e-5):
        rid = ohss.row_id(Z2, thr, 20 + 10)
        e = np.linalg.norm(Z2 - rid.U @ Z2[rid.skel])
        assert abs(e - rid.resid) <= 1e-10 * np.linalg.norm(Z2)
        sv = np.linalg.svd(Z2, compute_uv=False)
        assert e >= np.sqrt(np.sum(sv[rid.k:] ** 2)) * (1 - 1e-9)
        assert e <= thr


def _kahan(n, c, cplx=False):
    """Kahan's matrix diag(s^i) (I - c * strict upper ones), s^2 + c^2 = 1, with
    columns scaled by (1 - 1e-6)^j so that column pivoting keeps the natural
    order; complex: unit-modulus phases on the off-diagonal entries."""
    s = np.sqrt(1 - c * c)
    R = np.triu(-c * np.ones((n, n)), 1) + np.eye(n)
    if cplx:
        ph = np.exp(1j * 0.7 * np.subtract.outer(np.arange(n), np.arange(n)))
        R = np.where(np.eye(n, dtype=bool), 1.0, R * ph)
    return np.diag(s ** np.arange(n)) @ R @ np.diag((1 - 1e-6) ** np.arange(n))


@pytest.mark.parametrize("n,c,k,cplx", [(10, 0.6, 9, False), (10, 0.6, 9, True), (30, 0.285, 29, False),
                                        (24, 0.5, 20, True)])
def test_row_id_strong_rrqr_swaps_bound_p(n, c, k, cplx):
    C = _kahan(n, c, cplx)
    Z = C.T.copy()                     # row ID of Z = column ID of C
    _, R, perm = sla.qr(C, mode="economic", pivoting=True)
    T0 = sla.solve_triangular(R[:k, :k], R[:k, k:])
    assert np.max(np.abs(T0)) > 2.0    # column pivoting alone breaks the bound on P
    # a threshold between ||R[k:, k:]|| and ||R[k-1:, k-1:]|| selects rank k
    thr = 0.5 * (np.linalg.norm(R[k:, k:]) + np.linalg.norm(R[k - 1:, k - 1:]))
    rid = ohss.row_id(Z, thr, n)
    assert rid.k == k and rid.swaps >= 1
    assert rid.tmax <= 2.0
    J = rid.skel
    Jc = np.setdiff1d(np.arange(n), J)
    assert np.allclose(rid.U[J], np.eye(k), atol=0)
    assert np.max(np.abs(rid.U[Jc])) <= 2.0
    # T is the least-squares interpolation of the free columns by the skeleton
    Tls = np.linalg.lstsq(C[:, J], C[:, Jc], rcond=None)[0]
    assert np.allclose(rid.U[Jc].T, Tls, rtol=0, atol=1e-10 * max(1.0, np.abs(Tls).max()))
    # error identity with the final skeleton, and the determinant growth
    e = np.linalg.norm(Z - rid.U @ Z[J])
    assert abs(e - rid.resid) <= 1e-12 * np.linalg.norm(Z)
    assert e >= np.sqrt(np.sum(np.linalg.svd(Z, compute_uv=False)[k:] ** 2)) * (1 - 1e-9)
    d0 = abs(np.prod(np.diag(R[:k, :k])))
    d1 = abs(np.prod(np.diag(np.linalg.qr(C[:, J], mode="r"))))
    assert d1 > d0 * 2.0 ** rid.swaps


def test_row_id_without_large_coefficients_takes_no_swap():
    rng = np.random.default_rng(12)
    Z = rng.standard_normal((30, 40)) * np.logspace(0, -8, 30)[:, None]
    rid = ohss.row_id(Z, 1e-4 * np.linalg.norm(Z), 40)
    _, R, perm = sla.qr(Z.T, mode="economic", pivoting=True)
    T0 = sla.solve_triangular(R[:rid.k, :rid.k], R[:rid.k, rid.k:])
    if np.max(np.abs(T0)) <= 2.0:
        assert rid.swaps == 0 and np.array_equal(np.sort(rid.skel), np.sort(perm[:rid.k]))


def _kernel_matrix(n, cplx=False):
    x = np.sort(np.random.default_rng(3).uniform(0, 1, n))
    K = 1.0 / (1.0 + 30.0 * np.abs(x[:, None] - x[None, :]))
    if cplx:
        K = K * np.exp(1j * 5.0 * np.abs(x[:, None] - x[None, :]))
    return K


@pytest.mark.parametrize("cplx", [False, True])
def test_hss_compress_pins(cplx):
    from oracle.sets import hss_tree
    q = 4
    S = _kernel_matrix(40 * q, cplx)
    tree = hss_tree(40, 15, q)
    # tol -> 0: S reproduced
    log0 = ohss.compress_adaptive(S, tree, 0.0, None, 32)
    assert np.array_equal(log0.result.S_tilde, S)
    for tol in (1e-3, 1e-6):
        om = lambda l: philox.gaussian_matrix(11, 5, S.shape[0], l, cplx)
        log = ohss.compress_adaptive(S, tree, tol, om, 16)
        St = log.result.S_tilde
        assert not log.fell_back
        assert np.linalg.norm(S - St) <= tol * np.linalg.norm(S)
        # off-diagonal blocks of siblings have rank <= the left child's ID rank
        nodes = hss_postorder(tree)
        for t in nodes:
            if t.is_leaf:
                assert np.array_equal(St[t.lo:t.hi, t.lo:t.hi], S[t.lo:t.hi, t.lo:t.hi])
                continue
            a, b = t.left, t.right
            blk = St[a.lo:a.hi, b.lo:b.hi]
            sv = np.linalg.svd(blk, compute_uv=False)
            rank = int(np.sum(sv > 1e-12 * sv[0]))
            assert rank <= min(a.hi - a.lo, b.hi - b.lo, max(log.result.ranks))
    # smaller tol never lowers the largest rank
    r3 = ohss.compress_adaptive(S, tree, 1e-3, om, 16).result.max_rank
    r6 = ohss.compress_adaptive(S, tree, 1e-6, om, 16).result.max_rank
    assert r6 >= r3


def test_gmres_identity_preconditioner_textbook():
    rng = np.random.default_rng(4)
    n = 12
    A = rng.standard_normal((n, n)) + n * np.eye(n) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 0j
    res = og.gmres(lambda v: A @ v, lambda v: v, b, tol=1e-12, restart=n)
    assert res.iters <= n
    assert np.linalg.norm(res.x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(res.x)
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-14)      # minimal residual: non-increasing in a cycle
    # Givens: closed form zeroes the second entry and keeps the norm
    for a, bb in ((3 + 1j, -2 + 5j), (0j, 1 - 1j), (2.0, 0.0)):
        c, s = og.givens(a, bb)
        top = c * a + s * bb
        bot = -np.conj(s) * a + c * bb
        assert abs(bot) < 1e-14 and abs(abs(top) - np.hypot(abs(a), abs(bb))) < 1e-14


@pytest.mark.parametrize("cplx", [False, True])
def test_gmres_restart_cycles_are_least_squares_minimisers(cplx):
    rng = np.random.default_rng(13)
    n, m, cycles = 40, 5, 4
    A = np.diag(np.linspace(1.0, 8.0, n)) + 1.5 * np.triu(rng.standard_normal((n, n)), 1) / np.sqrt(n)
    Minv = np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    if cplx:
        A = A + 0.5j * np.diag(rng.standard_normal(n))
        Minv = Minv + 0.1j * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    res = og.gmres(lambda v: A @ v, lambda v: Minv @ v, b, tol=1e-15, restart=m, maxit=m * cycles)
    assert res.iters == m * cycles and res.restarts == cycles and not res.converged
    # independent: x_{c+1} = x_c + M^{-1} Q y, Q an orthonormal basis of K_m(A M^{-1}, r_c),
    # y the least-squares minimiser of ||r_c - A M^{-1} Q y||
    x = np.zeros(n, dtype=res.x.dtype)
    AM = A @ Minv
    for c in range(cycles):
        r = b - A @ x
        K = np.empty((n, m), dtype=res.x.dtype)
        K[:, 0] = r / np.linalg.norm(r)
        for j in range(1, m):
            w = AM @ K[:, j - 1]
            K[:, j] = w / np.linalg.norm(w)
        Q = np.linalg.qr(K)[0]
        y = np.linalg.lstsq(AM @ Q, r, rcond=None)[0]
        x = x + Minv @ (Q @ y)
        # the rotated residual at the cycle's last step is the true residual there
        assert abs(res.history[m * (c + 1) - 1] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) <= 1e-9
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)
    assert abs(res.true_relres - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) <= 1e-9


def test_gmres_zero_rhs_returns_zero():
    A = np.eye(4) * 2.0
    res = og.gmres(lambda v: A @ v, lambda v: v, np.zeros(4), tol=1e-8, x0=np.ones(4))
    assert res.iters == 0 and np.array_equal(res.x, np.zeros(4)) and res.true_relres == 0.0


def test_mlp_gradients_central_differences():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((16, 8))
    t = rng.standard_normal(16)
    params = omlp.init_params(3)
    loss, grads = omlp.loss_and_grad(params, X, t)
    h = 1e-6
    for pi in range(len(params)):
        P = params[pi]
        idx = [tuple(rng.integers(0, s) for s in P.shape) for _ in range(4)]
        for ix in idx:
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[pi][ix] += h
            pm[pi][ix] -= h
            fd = (omlp.loss_and_grad(pp, X, t)[0] - omlp.loss_and_grad(pm, X, t)[0]) / (2 * h)
            assert abs(fd - grads[pi][ix]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    params = omlp.init_params(1)
    grads = [np.full_like(p, 0.3) * np.sign(np.arange(p.size).reshape(p.shape) % 2 - 0.5)
             for p in params]
    new = omlp.adam_step(params, grads, {}, lr=0.01)
    for p, g, q in zip(params, grads, new):
        assert np.allclose(q - p, -0.01 * np.sign(g), rtol=1e-6, atol=0)


def test_preconditioned_gmres_poisson16_small_count():
    P = configs.make("poisson_p1_16")
    F = OracleFactor(P.op, P.tree, P.tol, seed=P.seed)
    assert F.max_err() <= P.tol
    res = og.gmres(F.matvec, F.apply, P.rhs[:, 0], tol=P.gmres_tol, restart=30)
    assert res.converged and res.iters <= 6
