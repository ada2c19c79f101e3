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

    def xface(X):   # face normal to x: traces vary along j (y)
        return np.kron(M1, X)

    def yface(X):   # face normal to y: traces vary along i (x)
        return np.kron(X, M1)

    # Interior-face blocks for a face with unit normal pointing from the
    # minus side (value trace e_m, derivative trace d_m along the normal)
    # to the plus side.  jump [u] = u- - u+, average {a du/dn}.
    def face_blocks(am, ap, sig, em, dm, ep, dp, scale_d):
        # scale_d: the 1/h of the normal derivative times the face length h = 1
        js = {0: 1.0, 1: -1.0}
        e = {0: em, 1: ep}
        d = {0: dm * scale_d, 1: dp * scale_d}
        a = {0: am, 1: ap}
        out = {}
        for s in (0, 1):          # test side (row)
            for t in (0, 1):      # trial side (col)
                X = (-(a[t] / 2.0) * js[s] * np.outer(e[s], d[t])
                     - (a[s] / 2.0) * js[t] * np.outer(d[s], e[t])
                     + sig * h * js[s] * js[t] * np.outer(e[s], e[t]))
                out[(s, t)] = X
        return out

    blocks: dict[tuple[int, int], np.ndarray] = {}

    def add(r, c, B):
        if (r, c) in blocks:
            blocks[(r, c)] = blocks[(r, c)] + B
        else:
            blocks[(r, c)] = B.astype(dt, copy=True)

    for ey in range(n):
        for ex in range(n):
            e = ex + n * ey
            a = coef[ey, ex]
            V = a * (ax * Kx + ay * Ky)
            if pde == "helmholtz":
                V = V - kappa * kappa * Mv
            elif reaction != 0.0:
                V = V + reaction * Mv
            add(e, e, V)

    # vertical faces (normal +x): between (ex, ey) and (ex+1, ey)
    for ey in range(n):
        for ex in range(n - 1):
            m = ex + n * ey
            pl = m + 1
            am, ap = coef[ey, ex] * ax, coef[ey, ex + 1] * ax
            sig = sig0 * max(coef[ey, ex], coef[ey, ex + 1])
            fb = face_blocks(am, ap, sig, e1, d1, e0, d0, 1.0)
            add(m, m, xface(fb[(0, 0)]))
            add(m, pl, xface(fb[(0, 1)]))
            add(pl, m, xface(fb[(1, 0)]))
            add(pl, pl, xface(fb[(1, 1)]))
    # horizontal faces (normal +y): between (ex, ey) and (ex, ey+1)
    for ey in range(n - 1):
        for ex in range(n):
            m = ex + n * ey
            pl = m + n
            am, ap = coef[ey, ex] * ay, coef[ey + 1, ex] * ay
            sig = sig0 * max(coef[ey, ex], coef[ey + 1, ex])
            fb = face_blocks(am, ap, sig, e1, d1, e0, d0, 1.0)
            add(m, m, yface(fb[(0, 0)]))
            add(m, pl, yface(fb[(0, 1)]))
            add(pl, m, yface(fb[(1, 0)]))
            add(pl, pl, yface(fb[(1, 1)]))

    # domain-boundary faces
    def bnd(e, c, a, ev, dv, normal_sign, face):
        # c: element coefficient (penalty scale), a: coefficient along the normal
        if pde == "helmholtz":
            X = -1j * kappa * h * np.outer(ev, ev)
        else:
            sig = sig0 * c
            dd = normal_sign * dv
            X = -a * np.outer(ev, dd) - a * np.outer(dd, ev) + sig * h * np.outer(ev, ev)
        add(e, e, xface(X) if face in "lr" else yface(X))

    for ey in range(n):
        bnd(0 + n * ey, coef[ey, 0], coef[ey, 0] * ax, e0, d0, -1.0, "l")
        bnd(n - 1 + n * ey, coef[ey, n - 1], coef[ey, n - 1] * ax, e1, d1, +1.0, "r")
    for ex in range(n):
        bnd(ex, coef[0, ex], coef[0, ex] * ay, e0, d0, -1.0, "b")
        bnd(ex + n * (n - 1), coef[n - 1, ex], coef[n - 1, ex] * ay, e1, d1, +1.0, "t")

    n_el = n * n
    rows: list[list[int]] = [[] for _ in range(n_el)]
    for (r, c) in blocks:
        rows[r].append(c)
    row_ptr = np.zeros(n_el + 1, dtype=np.int32)
    col_idx = []
    vals = []
    for r in range(n_el):
        cs = sorted(rows[r])
        row_ptr[r + 1] = row_ptr[r] + len(cs)
        for c in cs:
            col_idx.append(c)
            vals.append(blocks[(r, c)].T)  # store column-major
    return BlockOperator(n=n, p=p, q=q, row_ptr=row_ptr,
                         col_idx=np.asarray(col_idx, dtype=np.int32),
                         vals=np.ascontiguousarray(np.asarray(vals, dtype=dt)), h=h)


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
