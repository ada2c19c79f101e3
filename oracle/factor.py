"""Approximate LDM^t factorization and its inverse (oracle side).

Algorithm 2 (Section 3.2): at the leaves form S = A_bb - A_bi A_ii^{-1} A_ib
directly and compress it; then level by level form the merged blocks of
equation (32) from the children's compressed complements and the coupling
blocks A(B^mu, B^nu), eliminate I^ hat and compress the new complement.
The forest's two top boxes meet in the dense root block of equation (36),
factorized directly. The inverse M^{-t} D^{-1} L^{-1} (end of Section 3.2)
is applied by a forward sweep over the Gauss transforms, the block
diagonal solve, and a backward sweep.

Nodes are processed in height waves (leaves first), which in exact
arithmetic gives the same factors as the paper's level-by-level loop.
Each S is symmetrised, S <- (S + S^T)/2, before compression: the operators
here are symmetric or complex symmetric, so the basis of the columns is
taken equal to that of the rows.

Dense LU with partial pivoting (LAPACK getrf through SciPy) is the factor of
every A^_ii and of the root.

Test infrastructure only.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import hss, philox
from .sets import TreeSets


def csr_of(op) -> sp.csr_matrix:
    """Assemble the element blocks into a SciPy CSR matrix (for extraction)."""
    q = op.q
    data = np.transpose(op.vals, (0, 2, 1))
    return sp.bsr_matrix((data, op.col_idx, op.row_ptr),
                         shape=(op.ndof, op.ndof)).tocsr()


def dense_block(Acsr, rows, cols):
    return Acsr[rows][:, cols].toarray()


@dataclasses.dataclass
class NodeFactor:
    node: int
    idof: np.ndarray
    bdof: np.ndarray
    lu: tuple | None
    Aib: np.ndarray
    Abi: np.ndarray
    S: np.ndarray               # uncompressed complement
    S_tilde: np.ndarray         # compressed complement
    log: object                 # hss.CompressLog


class OracleFactor:
    def __init__(self, op, tree, tol: float, seed: int = 1508, l0: int = 32,
                 l_init: dict | None = None, symmetrize: bool = True, hss_leaf_elems: int = 4):
        self.op = op
        self.tol = tol
        self.seed = seed
        self.sets = TreeSets(op.row_ptr, op.col_idx, op.q, tree, hss_leaf_elems)
        self.A = csr_of(op)
        self.cplx = op.is_complex
        self.nodes: dict[int, NodeFactor] = {}
        t0 = time.perf_counter()
        for s in self.sets.elimination_order():
            ns = self.sets.sets[s]
            if ns.is_leaf:
                I, B = ns.idof, ns.bdof
                Aii = dense_block(self.A, I, I)
                Aib = dense_block(self.A, I, B)
                Abi = dense_block(self.A, B, I)
                Abb = dense_block(self.A, B, B)
            else:
                Ahat, U = self._merged(s)
                pos = {int(d): i for i, d in enumerate(U)}
                ii = np.array([pos[int(d)] for d in ns.idof], dtype=np.int64)
                bb = np.array([pos[int(d)] for d in ns.bdof], dtype=np.int64)
                Aii = Ahat[np.ix_(ii, ii)]
                Aib = Ahat[np.ix_(ii, bb)]
                Abi = Ahat[np.ix_(bb, ii)]
                Abb = Ahat[np.ix_(bb, bb)]
            if Aii.shape[0] > 0:
                lu = sla.lu_factor(Aii)
                S = Abb - Abi @ sla.lu_solve(lu, Aib)
            else:
                lu = None
                S = Abb.copy()
            if symmetrize:
                S = 0.5 * (S + S.T)
            l_start = l0 if l_init is None else int(l_init.get(s, l0))
            nb = S.shape[0]
            log = hss.compress_adaptive(
                S, ns.hss, tol,
                lambda l, s=s, nb=nb: philox.gaussian_matrix(seed, s, nb, l, self.cplx), l_start)
            self.nodes[s] = NodeFactor(s, ns.idof, ns.bdof, lu, Aib, Abi, S,
                                       log.result.S_tilde, log)
        # root (virtual node 1): equation (36)
        R, U = self._merged(1)
        self.root_idof = U
        self.root_lu = sla.lu_factor(R)
        self.root = R
        self.factor_seconds = time.perf_counter() - t0

    def _merged(self, s):
        """Dense merged matrix over [B^mu ; B^nu] for node s (equation (32) / (36))."""
        mu, nu = self.nodes[2 * s], self.nodes[2 * s + 1]
        Bm, Bn = mu.bdof, nu.bdof
        U = np.concatenate([Bm, Bn])
        nm = Bm.size
        M = np.zeros((U.size, U.size), dtype=mu.S_tilde.dtype)
        M[:nm, :nm] = mu.S_tilde
        M[nm:, nm:] = nu.S_tilde
        M[:nm, nm:] = dense_block(self.A, Bm, Bn)
        M[nm:, :nm] = dense_block(self.A, Bn, Bm)
        return M, U

    # ---- the inverse factorization ----
    def apply(self, x: np.ndarray) -> np.ndarray:
        """y = M^{-t} D^{-1} L^{-1} x (x: [ndof] or [ndof, nrhs])."""
        dt = np.result_type(x.dtype, self.root.dtype)
        r = np.array(x, dtype=dt, copy=True)
        order = self.sets.elimination_order()
        for s in order:                                   # L^{-1}, then D^{-1} on I^
            nf = self.nodes[s]
            if nf.lu is None:
                continue
            t = sla.lu_solve(nf.lu, r[nf.idof])
            r[nf.idof] = t
            r[nf.bdof] -= nf.Abi @ t
        r[self.root_idof] = sla.lu_solve(self.root_lu, r[self.root_idof])
        for s in reversed(order):                         # M^{-t}
            nf = self.nodes[s]
            if nf.lu is None:
                continue
            r[nf.idof] -= sla.lu_solve(nf.lu, nf.Aib @ r[nf.bdof])
        return r

    def matvec(self, x):
        return self.A @ x

    # ---- diagnostics ----
    def ranks(self):
        return {s: nf.log.result.max_rank for s, nf in self.nodes.items()}

    def max_err(self):
        return max((nf.log.result.err for nf in self.nodes.values()), default=0.0)
