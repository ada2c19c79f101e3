"""Right-preconditioned restarted GMRES(m) (oracle side).

The preconditioner is used inside GMRES (Introduction; Section 4). The
paper gives no further detail, so this is the textbook method (Saad and
Schultz 1986): Arnoldi with modified Gram-Schmidt on A M^{-1}, Hermitian
inner products, Givens rotations on the Hessenberg matrix, x0 = 0.
A cycle stops when the rotated residual |g_{j+1}| <= tol ||b||; the true
residual ||b - A x|| / ||b|| is then checked and the method restarts from x
if it is not below tol. The iteration count is the number of Arnoldi steps.

Test infrastructure only.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    restarts: int
    true_relres: float
    converged: bool
    history: list


def givens(a, b):
    """(c, s) with c real such that [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 * a
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    r = np.hypot(abs(a), abs(b))
    c = abs(a) / r
    s = (a / abs(a)) * np.conj(b) / r
    return c, s


def gmres(matvec, precond, b, tol=1e-8, restart=30, maxit=1000, x0=None) -> GmresResult:
    dt = np.result_type(b.dtype, np.float64)
    n = b.size
    x = np.zeros(n, dtype=dt) if x0 is None else np.array(x0, dtype=dt)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return GmresResult(np.zeros(n, dtype=dt), 0, 0, 0.0, True, [])
    iters = 0
    restarts = 0
    history = []
    while iters < maxit:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return GmresResult(x, iters, restarts, beta / bnorm, True, history)
        m = restart
        V = np.zeros((n, m + 1), dtype=dt)
        H = np.zeros((m + 1, m), dtype=dt)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=dt)
        g = np.zeros(m + 1, dtype=dt)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            z = precond(V[:, j])
            w = matvec(z)
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
            c, s = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            iters += 1
            j_done = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or iters >= maxit:
                break
        yk = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + precond(V[:, :j_done] @ yk)
        restarts += 1
    r = b - matvec(x)
    rel = np.linalg.norm(r) / bnorm
    return GmresResult(x, iters, restarts, rel, rel <= tol, history)
