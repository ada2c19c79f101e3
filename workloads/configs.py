"""Seeded synthetic workloads with the shapes of the paper's experiments.

Every input is generated here, on the host, from a seed; both the oracle
and the library consume the result. Nothing in this module computes any
part of the preconditioner.

Workloads (sizes follow the experiment settings of Section 4 scaled to the
problem sizes this project measures):
  poisson_p1_16       Poisson, p=1, 16x16 elements (1,024 dofs), Dirichlet,
                      ID tol 1e-6, FP64, rhs N(0,1), GMRES(30) to 1e-10.
  helmholtz_p2_64     Helmholtz, impedance BC, p=2, 64x64 (36,864 dofs),
                      8 dofs per wavelength, ID tol 1e-4, point source,
                      FP32 factor / FP64 GMRES to 1e-8.
  varpoisson_p3_128   -div(a grad u), a = exp(Gaussian random field,
                      squared-exponential covariance, length 0.1, var 1),
                      p=3, 128x128 (262,144 dofs), ID tol 1e-5, rhs N(0,1),
                      BF16 Schur products, GMRES to 1e-8.
  helmholtz_batch64   64 impedance Helmholtz problems, n ~ U{32..96}, p=2,
                      6-10 dofs per wavelength, 4 point sources each.
  helmholtz_p4_256    Helmholtz, p=4, 256x256 (1,638,400 dofs), 10 dofs
                      per wavelength, ID tol 1e-4.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import partition, sipg

BASE_SEED = 1508


@dataclasses.dataclass
class Problem:
    name: str
    op: sipg.BlockOperator
    tree: partition.Tree
    rhs: np.ndarray           # [ndof, nrhs]
    tol: float                # ID tolerance
    gmres_tol: float
    restart: int
    prec: str                 # "fp64" | "fp32" | "bf16"
    kappa: float
    coef: np.ndarray          # per-element coefficient [n, n]
    seed: int


def dofs_per_wavelength_kappa(n: int, p: int, dpw: float) -> float:
    """kappa such that one wavelength spans ``dpw`` DG nodes along an axis."""
    return 2.0 * math.pi * n * (p + 1) / dpw


def grf(n: int, length: float, var: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian random field at element centroids, covariance
    var * exp(-r^2 / (2 length^2)), sampled exactly through the Kronecker
    structure of the covariance on a tensor grid."""
    xc = (np.arange(n) + 0.5) / n
    C1 = np.exp(-(xc[:, None] - xc[None, :]) ** 2 / (2.0 * length * length))
    lam, Q = np.linalg.eigh(C1)
    lam = np.clip(lam, 0.0, None)
    xi = rng.standard_normal((n, n))
    S = np.sqrt(np.outer(lam, lam)) * xi
    G = Q @ S @ Q.T
    return math.sqrt(var) * G


def make(name: str, *, n: int | None = None, p: int | None = None, seed_offset: int = 0,
         nrhs: int = 1, leaf_elems: int = 16, scheme: str = "boxes") -> Problem:
    """Build a named workload. ``n``/``p`` override the grid for reduced-size
    variants of the same problem family (used by the parity tests)."""
    if name.startswith("poisson_p1"):
        idx, n0, p0, pde = 0, 16, 1, "poisson"
        tol, gtol, prec, rhs_kind = 1e-6, 1e-10, "fp64", "normal"
    elif name.startswith("helmholtz_p2"):
        idx, n0, p0, pde = 1, 64, 2, "helmholtz"
        tol, gtol, prec, rhs_kind = 1e-4, 1e-8, "fp32", "point"
    elif name.startswith("varpoisson_p3"):
        idx, n0, p0, pde = 2, 128, 3, "varpoisson"
        tol, gtol, prec, rhs_kind = 1e-5, 1e-8, "bf16", "normal"
    elif name.startswith("helmholtz_p4"):
        idx, n0, p0, pde = 4, 256, 4, "helmholtz"
        tol, gtol, prec, rhs_kind = 1e-4, 1e-8, "fp32", "point"
    else:
        raise KeyError(name)
    n = n0 if n is None else n
    p = p0 if p is None else p
    seed = BASE_SEED + idx + 1000 * seed_offset
    rng = np.random.default_rng(seed)
    coef = np.ones((n, n))
    kappa = 0.0
    if pde == "helmholtz":
        dpw = 10.0 if idx == 4 else 8.0
        kappa = dofs_per_wavelength_kappa(n, p, dpw)
        op = sipg.assemble(n, p, "helmholtz", kappa=kappa)
    elif pde == "varpoisson":
        coef = np.exp(grf(n, 0.1, 1.0, np.random.default_rng(seed + 7)))
        op = sipg.assemble(n, p, "poisson", coef=coef)
    else:
        op = sipg.assemble(n, p, "poisson")
    tree = partition.build_tree(n, n, leaf_elems=leaf_elems, scheme=scheme)
    if rhs_kind == "normal":
        b = rng.standard_normal((op.ndof, nrhs))
    else:
        cols = []
        for _ in range(nrhs):
            x0, y0 = rng.uniform(0.0, 1.0, size=2)
            cols.append(sipg.point_source(n, p, x0, y0))
        b = np.stack(cols, axis=1)
    if op.is_complex:
        b = b.astype(np.complex128)
    return Problem(name=name, op=op, tree=tree, rhs=b, tol=tol, gmres_tol=gtol,
                   restart=30, prec=prec, kappa=kappa, coef=coef, seed=seed)


# Problem families of the paper's Section 4 studies, for the h/p sweeps and the
# partition studies (all real, homogeneous Dirichlet data, FP64):
#   poisson   -lap u = f                                   (Poisson study)
#   cavity    -lap u - kappa^2 u = f, the soft cavity        (Helmholtz study)
#   aniso     -u_xx - a0 u_yy + c0 u = f (equation (60) normalized by a11)
#   contrast  -div(rho^-1 grad u) - kappa^2 u = f, rho = rho_d in the rectangular
#             enclosure D = [0.125, 0.875] x [0.375, 0.5] of the partition
#             figure, 1 elsewhere (per element, by its centroid)
# kappa keeps `dpw` DG nodes per wavelength along an axis as n and p vary: the
# stand-in for the paper's constant dispersion error.
STUDY_TOL = {"poisson": 1e-3, "cavity": 1e-3, "aniso": 1e-3, "contrast": 1e-3}


def contrast_coef(n: int, rho_d: float) -> np.ndarray:
    """rho^-1 per element ([ey, ex]) with rho = rho_d in the enclosure D."""
    xc = (np.arange(n) + 0.5) / n
    inside = ((xc[None, :] > 0.125) & (xc[None, :] < 0.875) & (xc[:, None] > 0.375) & (xc[:, None] < 0.5))
    return np.where(inside, 1.0 / rho_d, 1.0)


def study(kind: str, n: int, p: int, *, scheme: str = "boxes", a0: float = 1e-6, c0: float = 1.0,
          rho_d: float = 1e3, dpw: float = 8.0, leaf_elems: int = 16, seed_offset: int = 0,
          tol: float | None = None) -> Problem:
    """One problem of a Section 4 study family (see above), rhs N(0, 1), ID tol
    STUDY_TOL (or ``tol``), GMRES(30) to 1e-8, FP64."""
    if kind not in STUDY_TOL:
        raise KeyError(kind)
    seed = BASE_SEED + 10 + ["poisson", "cavity", "aniso", "contrast"].index(kind) + 1000 * seed_offset
    rng = np.random.default_rng(seed)
    coef = np.ones((n, n))
    kappa = 0.0
    if kind == "poisson":
        op = sipg.assemble(n, p, "poisson")
    elif kind == "cavity":
        kappa = dofs_per_wavelength_kappa(n, p, dpw)
        op = sipg.assemble(n, p, "poisson", reaction=-kappa * kappa)
    elif kind == "aniso":
        op = sipg.assemble(n, p, "poisson", aniso=(1.0, a0), reaction=c0)
    else:
        kappa = dofs_per_wavelength_kappa(n, p, dpw)
        coef = contrast_coef(n, rho_d)
        op = sipg.assemble(n, p, "poisson", coef=coef, reaction=-kappa * kappa)
    tree = partition.build_tree(n, n, leaf_elems=leaf_elems, scheme=scheme)
    b = rng.standard_normal((op.ndof, 1))
    return Problem(name=f"{kind}_p{p}_{n}_{scheme}", op=op, tree=tree, rhs=b,
                   tol=STUDY_TOL[kind] if tol is None else tol,
                   gmres_tol=1e-8, restart=30, prec="fp64", kappa=kappa, coef=coef, seed=seed)


def make_batch(count: int = 64, n_lo: int = 32, n_hi: int = 96, p: int = 2,
               nrhs: int = 4, seed_offset: int = 0) -> list[Problem]:
    """The batched Helmholtz workload: ``count`` problems of uneven size."""
    seed = BASE_SEED + 3 + 1000 * seed_offset
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        dpw = float(rng.uniform(6.0, 10.0))
        kappa = dofs_per_wavelength_kappa(n, p, dpw)
        op = sipg.assemble(n, p, "helmholtz", kappa=kappa)
        tree = partition.build_tree(n, n, leaf_elems=16)
        cols = []
        for _ in range(nrhs):
            x0, y0 = rng.uniform(0.0, 1.0, size=2)
            cols.append(sipg.point_source(n, p, x0, y0))
        b = np.stack(cols, axis=1).astype(np.complex128)
        out.append(Problem(name=f"helmholtz_batch_{i}", op=op, tree=tree, rhs=b, tol=1e-4,
                           gmres_tol=1e-8, restart=30, prec="fp32", kappa=kappa,
                           coef=np.ones((n, n)), seed=seed * 100 + i))
    return out
