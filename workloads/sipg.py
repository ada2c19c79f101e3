"""Symmetric interior-penalty DG (SIPG) on a uniform n x n grid of squares.

This module only manufactures the test matrices: it is the discretisation
that feeds the preconditioner, not part of the preconditioner. The paper
builds its examples from interior-penalty nodal DG on the unit square
(Section 4, first paragraph); here the elements are squares with
tensor-product Lagrange bases on Gauss-Lobatto nodes.

Operators (Section 4):
  * Poisson / variable-coefficient Poisson  -div(a grad u) = f, a constant
    per element, homogeneous Dirichlet data imposed weakly (Nitsche).
  * Helmholtz  -lap u - kappa^2 u = f with the impedance condition
    du/dn - i kappa u = 0 (the weak form gains -i kappa * boundary mass),
    giving a complex-symmetric matrix.

Layout of the returned operator (block compressed rows, one block per
element pair): element e = ex + n*ey, q = (p+1)^2 dofs per element, dof
= e*q + (ix + (p+1)*iy). ``vals[b]`` is the q x q block stored column-major,
i.e. ``vals[b, c, r]`` holds A(row r, col c) of block b.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def gll_nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre nodes of degree p mapped to [0, 1]."""
    if p < 1:
        raise ValueError("p >= 1 required")
    if p == 1:
        x = np.array([-1.0, 1.0])
    else:
        c = np.zeros(p + 1)
        c[p] = 1.0
        dP = np.polynomial.legendre.legder(c)
        inner = np.sort(np.real(np.polynomial.legendre.legroots(dP)))
        x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def gauss_rule(nq: int):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


class Lagrange1D:
    """Lagrange basis on the GLL nodes, evaluated through its monomial form."""

    def __init__(self, p: int):
        self.p = p
        self.nodes = gll_nodes(p)
        V = np.vander(self.nodes, p + 1, increasing=True)
        self.coef = np.linalg.inv(V)  # coef[m, i]: x^m coefficient of l_i

    def value(self, x) -> np.ndarray:
        x = np.atleast_1d(np.asarray(x, dtype=float))
        P = np.vander(x, self.p + 1, increasing=True)
        return P @ self.coef  # [len(x), p+1]

    def deriv(self, x) -> np.ndarray:
        x = np.atleast_1d(np.asarray(x, dtype=float))
        m = np.arange(self.p + 1)
        P = np.zeros((x.size, self.p + 1))
        for k in range(1, self.p + 1):
            P[:, k] = k * x ** (k - 1)
        del m
        return P @ self.coef


@dataclasses.dataclass
class BlockOperator:
    """Element-block (BSR) operator. Never assembled as a dense matrix here."""

    n: int                      # elements per side
    p: int                      # polynomial degree
    q: int                      # dofs per element
    row_ptr: np.ndarray         # int32 [n_el + 1]
    col_idx: np.ndarray         # int32 [nnzb]
    vals: np.ndarray            # float64 or complex128 [nnzb, q, q] (column-major blocks)
    h: float

    @property
    def n_el(self) -> int:
        return self.n * self.n

    @property
    def ndof(self) -> int:
        return self.n_el * self.q

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.vals)

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A x with the element blocks (used by fixtures and tests)."""
        q = self.q
        X = x.reshape(self.n_el, q, *x.shape[1:])
        Y = np.zeros(X.shape, dtype=np.result_type(self.vals, x))
        for e in range(self.n_el):
            for b in range(self.row_ptr[e], self.row_ptr[e + 1]):
                blk = self.vals[b].T  # row-major view of the block
                Y[e] += blk @ X[self.col_idx[b]]
        return Y.reshape(x.shape)

    def to_dense(self) -> np.ndarray:
        q = self.q
        A = np.zeros((self.ndof, self.ndof), dtype=self.vals.dtype)
        for e in range(self.n_el):
            for b in range(self.row_ptr[e], self.row_ptr[e + 1]):
                c = self.col_idx[b]
                A[e * q:(e + 1) * q, c * q:(c + 1) * q] = self.vals[b].T
        return A

    def to_scipy(self):
        import scipy.sparse as sp
        q = self.q
        data = np.transpose(self.vals, (0, 2, 1))  # row-major blocks
        return sp.bsr_matrix((data, self.col_idx, self.row_ptr),
                             shape=(self.ndof, self.ndof)).tocsr()


def assemble(n: int, p: int, pde: str = "poisson", coef: np.ndarray | None = None,
             kappa: float = 0.0, penalty: float = 10.0,
             aniso: tuple[float, float] = (1.0, 1.0), reaction: float = 0.0) -> BlockOperator:
    """Assemble the SIPG operator on the unit square with n x n elements.

    pde = "poisson": -div(a grad u) + reaction*u, homogeneous Dirichlet (Nitsche).
          ``coef`` (n x n, indexed [ey, ex]) is the per-element coefficient a;
          ``aniso`` scales the x and y second derivatives (diag tensor).
    pde = "helmholtz": -lap u - kappa^2 u with du/dn - i kappa u = 0.
    Penalty sigma_F = penalty * p^2 / h * max(a-, a+) (one-sided on the boundary).
    """
    if pde not in ("poisson", "helmholtz"):
        raise ValueError(pde)
    h = 1.0 / n
    q = (p + 1) ** 2
    L = Lagrange1D(p)
    xq, wq = gauss_rule(p + 2)
    Bq = L.value(xq)
    Dq = L.deriv(xq)
    M1 = Bq.T @ (wq[:, None] * Bq)            # int_0^1 l_i l_j
    K1 = Dq.T @ (wq[:, None] * Dq)            # int_0^1 l_i' l_j'
    e0 = L.value(0.0)[0]
    e1 = L.value(1.0)[0]
    d0 = L.deriv(0.0)[0]
    d1 = L.deriv(1.0)[0]
    if coef is None:
        coef = np.ones((n, n))
    coef = np.asarray(coef, dtype=float)
    ax, ay = aniso
    sig0 = penalty * p * p / h

    cplx = pde == "helmholtz"
    dt = np.complex128 if cplx else np.float64
    # Volume term: x-derivatives act on index i (fast), y-derivatives on j.
    Kx = np.kron(M1, K1)        # [j*(p+1)+i, ...] = M1[j,j'] K1[i,i']
    Ky = np.kron(K1, M1)
    Mv = h * h * np.kron(M1, M1)

    # Interior-face blocks for a face with unit normal pointing from the minus
    # side (value trace e1, derivative trace d1 along the normal) to the plus
    # side (e0, d0): jump [u] = u- - u+, average {a du/dn}. Face matrices act on
    # the traces; a face normal to x spreads them with kron(M1, X), a face
    # normal to y with kron(X, M1).
    # Per-element and per-face scalars as arrays; every block entry is formed by
    # the same sequence of floating-point operations as a one-face-at-a-time
    # loop, and each element's diagonal block accumulates its contributions in
    # a fixed order: volume, left face, right face, lower face, upper face, then
    # the domain-boundary faces (left, right, bottom, top).
    def kron_faces(Mfix, X, normal_x):
        # np.kron(M1, X) (faces normal to x) or np.kron(X, M1) (normal to y) for a
        # stack of face matrices X [F, p+1, p+1]
        F = X.shape[0]
        if normal_x:
            K = Mfix[None, :, None, :, None] * X[:, None, :, None, :]
        else:
            K = X[:, :, None, :, None] * Mfix[None, None, :, None, :]
        return K.reshape(F, q, q)

    def face_stack(am, ap, sig, s, t):
        # block (test side s, trial side t) of every face; sides 0 = minus, 1 = plus
        js = {0: 1.0, 1: -1.0}
        e = {0: e1, 1: e0}
        d = {0: d1, 1: d0}
        a = {0: am, 1: ap}
        c1 = -(a[t] / 2.0) * js[s]
        c2 = (a[s] / 2.0) * js[t]
        c3 = sig * h * js[s] * js[t]
        return (c1[:, None, None] * np.outer(e[s], d[t])[None]
                - c2[:, None, None] * np.outer(d[s], e[t])[None]
                + c3[:, None, None] * np.outer(e[s], e[t])[None])

    # volume
    acoef = coef.reshape(-1)                                   # element e = ex + n*ey
    diag = acoef[:, None, None] * (ax * Kx + ay * Ky)[None]
    if pde == "helmholtz":
        diag = diag - (kappa * kappa * Mv)[None]
    elif reaction != 0.0:
        diag = diag + (reaction * Mv)[None]
    diag = diag.astype(dt).reshape(n, n, q, q)                # [ey, ex]
    right = up = None
    if n > 1:
        # vertical faces between (ex, ey) and (ex + 1, ey): arrays [n, n - 1] flattened
        am = (coef[:, :-1] * ax).reshape(-1)
        ap = (coef[:, 1:] * ax).reshape(-1)
        sig = sig0 * np.maximum(coef[:, :-1], coef[:, 1:]).reshape(-1)
        fx = {st: kron_faces(M1, face_stack(am, ap, sig, *st), True).reshape(n, n - 1, q, q)
              for st in ((0, 0), (0, 1), (1, 0), (1, 1))}
        # horizontal faces between (ex, ey) and (ex, ey + 1): arrays [n - 1, n]
        am = (coef[:-1, :] * ay).reshape(-1)
        ap = (coef[1:, :] * ay).reshape(-1)
        sig = sig0 * np.maximum(coef[:-1, :], coef[1:, :]).reshape(-1)
        fy = {st: kron_faces(M1, face_stack(am, ap, sig, *st), False).reshape(n - 1, n, q, q)
              for st in ((0, 0), (0, 1), (1, 0), (1, 1))}
        diag[:, 1:] += fx[(1, 1)]
        diag[:, :-1] += fx[(0, 0)]
        diag[1:, :] += fy[(1, 1)]
        diag[:-1, :] += fy[(0, 0)]
        right = (fx[(0, 1)], fx[(1, 0)])   # blocks (e, e+1) and (e+1, e)
        up = (fy[(0, 1)], fy[(1, 0)])      # blocks (e, e+n) and (e+n, e)

    # domain-boundary faces
    def bnd_stack(cvec, avec, ev, dv, normal_sign, normal_x):
        F = cvec.size
        if pde == "helmholtz":
            X = np.broadcast_to((-1j * kappa * h * np.outer(ev, ev))[None], (F, p + 1, p + 1))
        else:
            sig = sig0 * cvec
            dd = normal_sign * dv
            X = (-avec[:, None, None] * np.outer(ev, dd)[None]
                 - avec[:, None, None] * np.outer(dd, ev)[None]
                 + (sig * h)[:, None, None] * np.outer(ev, ev)[None])
        return kron_faces(M1, np.ascontiguousarray(X), normal_x)

    diag[:, 0] += bnd_stack(coef[:, 0], coef[:, 0] * ax, e0, d0, -1.0, True)
    diag[:, n - 1] += bnd_stack(coef[:, n - 1], coef[:, n - 1] * ax, e1, d1, +1.0, True)
    diag[0, :] += bnd_stack(coef[0, :], coef[0, :] * ay, e0, d0, -1.0, False)
    diag[n - 1, :] += bnd_stack(coef[n - 1, :], coef[n - 1, :] * ay, e1, d1, +1.0, False)

    # block rows in ascending column order: e - n, e - 1, e, e + 1, e + n
    n_el = n * n
    ey, ex = np.divmod(np.arange(n_el), n)
    has = [ey > 0, ex > 0, np.ones(n_el, bool), ex < n - 1, ey < n - 1]
    offs = [-n, -1, 0, 1, n]
    counts = np.sum(has, axis=0)
    row_ptr = np.zeros(n_el + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(counts)
    nnzb = int(row_ptr[-1])
    col_idx = np.empty(nnzb, dtype=np.int32)
    vals = np.empty((nnzb, q, q), dtype=dt)
    slot = row_ptr[:-1].astype(np.int64).copy()
    for k, (hk, off) in enumerate(zip(has, offs)):
        e = np.nonzero(hk)[0]
        if e.size == 0:
            continue
        pos = slot[e]
        col_idx[pos] = e + off
        eyk, exk = ey[e], ex[e]
        if off == 0:
            B = diag[eyk, exk]
        elif off == 1:
            B = right[0][eyk, exk]
        elif off == -1:
            B = right[1][eyk, exk - 1]
        elif off == n:
            B = up[0][eyk, exk]
        else:
            B = up[1][eyk - 1, exk]
        vals[pos] = np.transpose(B, (0, 2, 1))   # store column-major
        slot[e] += 1
    return BlockOperator(n=n, p=p, q=q, row_ptr=row_ptr, col_idx=col_idx,
                         vals=np.ascontiguousarray(vals), h=h)


def load_vector(n: int, p: int, f) -> np.ndarray:
    """b_j = int f phi_j by tensor Gauss quadrature (f vectorised in x, y)."""
    h = 1.0 / n
    L = Lagrange1D(p)
    xq, wq = gauss_rule(p + 3)
    Bq = L.value(xq)
    q = (p + 1) ** 2
    b = np.zeros(n * n * q)
    for ey in range(n):
        for ex in range(n):
            X = (ex + xq) * h
            Y = (ey + xq) * h
            F = f(X[None, :], Y[:, None])               # [qy, qx]
            W = (wq[:, None] * wq[None, :]) * h * h
            loc = Bq.T @ (W * F).T @ Bq                  # [i, j]
            e = ex + n * ey
            b[e * q:(e + 1) * q] = loc.T.reshape(-1)     # index j*(p+1)+i
    return b


def l2_error(n: int, p: int, u: np.ndarray, exact) -> float:
    """sqrt(sum_K int_K (u_h - u)^2) with a tensor Gauss rule."""
    h = 1.0 / n
    L = Lagrange1D(p)
    xq, wq = gauss_rule(p + 3)
    Bq = L.value(xq)
    q = (p + 1) ** 2
    err = 0.0
    for ey in range(n):
        for ex in range(n):
            e = ex + n * ey
            c = u[e * q:(e + 1) * q].reshape(p + 1, p + 1)   # [j, i]
            uh = Bq @ c @ Bq.T                              # [qy, qx]
            X = (ex + xq) * h
            Y = (ey + xq) * h
            ue = exact(X[None, :], Y[:, None])
            W = (wq[:, None] * wq[None, :]) * h * h
            err += float(np.sum(W * np.abs(uh - ue) ** 2))
    return float(np.sqrt(err))


def point_source(n: int, p: int, x0: float, y0: float) -> np.ndarray:
    """b_j = phi_j(x0, y0): the load of a unit point source."""
    h = 1.0 / n
    ex = min(int(x0 / h), n - 1)
    ey = min(int(y0 / h), n - 1)
    L = Lagrange1D(p)
    vx = L.value(x0 / h - ex)[0]
    vy = L.value(y0 / h - ey)[0]
    q = (p + 1) ** 2
    b = np.zeros(n * n * q)
    e = ex + n * ey
    b[e * q:(e + 1) * q] = np.outer(vy, vx).reshape(-1)
    return b
