"""Interpolative decomposition and HSS compression (oracle side).

Section 1 defines the HSS form (nested bases: the tall basis of a parent is
the block diagonal of its children's tall bases times a short basis) and
the interpolative decomposition A = A_skel P, where A_skel keeps k columns
of A and P contains the k x k identity, its entries preferably bounded by 2.
Theorem 1 builds an HSS approximant from products with random test
vectors (oversampling p = 10) plus individual entries.

The construction here, for a symmetric or complex-symmetric S (so the row
and column bases coincide and V = U), visits the HSS nodes children first:
  candidates R: all indices of a leaf, or the union of the children's
          skeletons J for an internal node (the nesting condition);
  samples   Z = S(R, complement of tau) Omega(complement of tau, :),
          formed as Y(R, :) - S(R, tau) Omega(tau, :) with Y = S Omega;
  row ID    CPQR of Z^T (column pivoting, Businger-Golub): keep the
          smallest k with ||R22||_F <= threshold; J = R[perm[:k]],
          T = R11^{-1} R12, U[perm[:k]] = I, U[perm[k:]] = T^T, so that
          Z ~= U Z(J, :).
  bounded P Section 1 asks for an interpolation matrix whose entries do not
          exceed 2 in modulus. While max |T| > 2 the skeleton column i and
          the free column j of the largest |T_ij| trade places (ties: the
          lowest skeleton position i, then the lowest candidate index of j;
          the incoming column takes position i) and T is formed again from
          a QR without pivoting of the reordered columns (Gu and Eisenstat's
          strong RRQR with f = 2). Every such swap multiplies |det R11| by at
          least |T_ij| > 2, so the loop ends; k does not change.
Generators: leaf diagonal blocks D = S(tau, tau); sibling blocks
B_ab = S(J_a, J_b). The approximant is S~(a, b) = Ut_a B_ab Ut_b^T with the
tall bases Ut (leaf: U; parent: diag(Ut_a, Ut_b) U).

Tolerance reading (the paper asks for ||A - A_HSS|| <= eps without naming
the norm): relative Frobenius error per node, ||S - S~||_F <= tol ||S||_F.
Per-ID threshold on the true block error: delta = tol ||S||_F / (4 sqrt(2 n_id));
on the samples it is delta * sqrt(l) (E||E Omega||_F^2 = l ||E||_F^2). The
sqrt(2 n_id) splits the budget between the IDs as if their errors added in
quadrature; the factor 1/4 allows for the nested bases, through which a
child's truncation error reaches the parent's block multiplied by the
parent's interpolation matrix (entries up to 2 in modulus). A node whose
measured error misses tol is redone with delta / 4; an ID that needs more
than l - p_os rows is redone with l doubled. A node whose measured error
meets tol is accepted as it is.

Test infrastructure only.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .sets import HssNode, hss_postorder

P_OS = 10
INITIAL_DELTA_SCALE = 0.25  # delta's first value relative to tol ||S||_F / sqrt(2 n_id)


@dataclasses.dataclass
class RowID:
    k: int
    skel: np.ndarray        # indices into the candidate list, pivot order
    U: np.ndarray           # |R| x k interpolation matrix
    resid: float            # ||R22||_F of the sampled matrix (after the swaps)
    exhausted: bool         # needed more rows than the samples can certify
    tmax: float             # max |T| (at most 2 after the swaps)
    swaps: int = 0          # strong-RRQR swaps taken


MAX_SWAPS = 64


def _tail_norms(R: np.ndarray) -> np.ndarray:
    """tail[k] = ||R[k:, k:]||_F for k = 0..r (tail[r] = 0: the remaining columns
    lie in the span of the first r)."""
    r = R.shape[0]
    tail = np.zeros(r + 1)
    for k in range(r - 1, -1, -1):
        tail[k] = np.sqrt(tail[k + 1] ** 2 + np.sum(np.abs(R[k, k:]) ** 2)
                          + np.sum(np.abs(R[k + 1:, k]) ** 2))
    return tail


def row_id(Z: np.ndarray, thresh: float, l: int) -> RowID:
    """Row interpolative decomposition of Z (|R| x l) by CPQR of Z^T, then the
    swaps that bound the interpolation coefficients by 2."""
    m = Z.shape[0]
    if m == 0:
        return RowID(0, np.zeros(0, dtype=np.int64), np.zeros((0, 0), Z.dtype), 0.0, False, 0.0)
    _, R, perm = sla.qr(Z.T, mode="economic", pivoting=True)
    tail = _tail_norms(R)
    k = next(kk for kk in range(R.shape[0] + 1) if tail[kk] <= thresh)
    exhausted = (k < m) and (k + P_OS > l)
    if k == 0:
        U = np.zeros((m, 0), dtype=Z.dtype)
        return RowID(0, np.zeros(0, dtype=np.int64), U, tail[0], exhausted, 0.0)
    T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
    resid = tail[k]
    swaps = 0
    while T.size and np.max(np.abs(T)) > 2.0 and swaps < MAX_SWAPS:
        aT = np.abs(T)
        ii, jj = np.nonzero(aT == aT.max())
        best = min(zip(ii.tolist(), jj.tolist()), key=lambda ij: (ij[0], perm[k + ij[1]]))
        i, j = best
        perm = perm.copy()
        perm[i], perm[k + j] = perm[k + j], perm[i]
        R = sla.qr(Z.T[:, perm], mode="economic")[1]
        T = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
        resid = float(np.linalg.norm(R[k:, k:]))
        swaps += 1
    U = np.zeros((m, k), dtype=np.result_type(Z.dtype, T.dtype))
    U[perm[:k], :] = np.eye(k)
    U[perm[k:], :] = T.T
    tmax = float(np.max(np.abs(T))) if T.size else 0.0
    return RowID(k, perm[:k].astype(np.int64), U, resid, exhausted, tmax, swaps)


@dataclasses.dataclass
class HssResult:
    S_tilde: np.ndarray
    err: float              # ||S - S~||_F / ||S||_F
    ranks: list             # rank of every ID, post-order
    max_rank: int
    exhausted: bool
    tmax: float
    n_id: int


def count_ids(t: HssNode) -> int:
    return len(hss_postorder(t)) - 1


def compress(S: np.ndarray, tree: HssNode, delta: float, Omega: np.ndarray) -> HssResult:
    """One pass of the randomized interpolative HSS construction (Theorem 1)
    with the per-ID true-error threshold ``delta`` and test matrix Omega (n x l)."""
    n = S.shape[0]
    l = Omega.shape[1]
    Y = S @ Omega
    order = hss_postorder(tree)
    skel: dict[int, np.ndarray] = {}      # id(node) -> skeleton indices into S
    U: dict[int, np.ndarray] = {}
    ranks = []
    exhausted = False
    tmax = 0.0
    thresh = delta * np.sqrt(l)
    for t in order:
        if t is tree:
            break
        if t.is_leaf:
            Rset = np.arange(t.lo, t.hi)
        else:
            Rset = np.concatenate([skel[id(t.left)], skel[id(t.right)]])
        Z = Y[Rset, :] - S[np.ix_(Rset, np.arange(t.lo, t.hi))] @ Omega[t.lo:t.hi, :]
        rid = row_id(Z, thresh, l)
        skel[id(t)] = Rset[rid.skel]
        U[id(t)] = rid.U
        ranks.append(rid.k)
        exhausted |= rid.exhausted
        tmax = max(tmax, rid.tmax)
    # tall bases, children first
    Ut: dict[int, np.ndarray] = {}
    for t in order:
        if t is tree:
            break
        if t.is_leaf:
            Ut[id(t)] = U[id(t)]
        else:
            a, b = Ut[id(t.left)], Ut[id(t.right)]
            D = np.zeros((a.shape[0] + b.shape[0], a.shape[1] + b.shape[1]), dtype=S.dtype)
            D[:a.shape[0], :a.shape[1]] = a
            D[a.shape[0]:, a.shape[1]:] = b
            Ut[id(t)] = D @ U[id(t)]
    St = np.zeros_like(S)
    for t in order:
        if t.is_leaf:
            St[t.lo:t.hi, t.lo:t.hi] = S[t.lo:t.hi, t.lo:t.hi]
        else:
            a, b = t.left, t.right
            B = S[np.ix_(skel[id(a)], skel[id(b)])]
            St[a.lo:a.hi, b.lo:b.hi] = Ut[id(a)] @ B @ Ut[id(b)].T
            B2 = S[np.ix_(skel[id(b)], skel[id(a)])]
            St[b.lo:b.hi, a.lo:a.hi] = Ut[id(b)] @ B2 @ Ut[id(a)].T
    nrm = np.linalg.norm(S)
    err = float(np.linalg.norm(S - St) / nrm) if nrm > 0 else 0.0
    return HssResult(St, err, ranks, max(ranks) if ranks else 0, exhausted, tmax, len(ranks))


@dataclasses.dataclass
class CompressLog:
    attempts: int
    l: int
    delta_scale: float
    result: HssResult
    fell_back: bool


def compress_adaptive(S: np.ndarray, tree: HssNode, tol: float, omega_fn, l0: int,
                      max_attempts: int = 8) -> CompressLog:
    """Randomized HSS compression with the judge / rank-growth loop.

    omega_fn(l) returns the node's n x l test matrix (its first columns do not
    depend on l). tol = 0 keeps S unchanged (exact factorization)."""
    n = S.shape[0]
    nrm = np.linalg.norm(S)
    n_id = count_ids(tree)
    if tol <= 0.0 or n_id == 0 or nrm == 0.0:
        return CompressLog(0, 0, 1.0, HssResult(S.copy(), 0.0, [], 0, False, 0.0, n_id), False)
    l_cap = n + P_OS
    l = min(l0, l_cap)
    scale = INITIAL_DELTA_SCALE
    res = None
    for att in range(1, max_attempts + 1):
        delta = scale * tol * nrm / np.sqrt(2.0 * n_id)
        res = compress(S, tree, delta, omega_fn(l))
        if res.err <= tol:
            return CompressLog(att, l, scale, res, False)
        if res.exhausted and l < l_cap:
            l = min(2 * l, l_cap)
        else:
            scale /= 4.0
    return CompressLog(max_attempts, l, scale,
                       HssResult(S.copy(), 0.0, res.ranks if res else [], 0, False, 0.0, n_id), True)
