"""The parameter studies of the paper's Section 4 on the GPU path.

    python experiments.py hp [--kinds poisson,cavity] [--ns 16,32,64,128] [--n-p 32]
                             [--ps 1,2,3,4] [--p-h 2] [--tol 1e-3] [--scale fixed|cond]
                             [--json FILE]
    python experiments.py partition [--n 32] [--p 1] [--tol 1e-3] [--json FILE]

hp: h-sweeps (p fixed, n elements per side doubling) and p-sweeps (n fixed) of
the Poisson problem and the Helmholtz soft cavity (Dirichlet data, kappa at a
fixed number of DG nodes per wavelength). Per run: GMRES(30) iterations to
1e-8; for the top-level box (heap id 2) its boundary size n_b, the largest ID
rank k of its compressed Schur complement and the final sample count l; and
the compression cost of every box from the ID cost estimate l k n log n
(Section 1, equation (43)) with the box's l, k and n = n_b, summed per level.
The summary fits, over each sweep, the growth of k with n_b and of the
top-level box's cost with N, the quantities of Figure 9 and equations (39)-(40)
and (56)-(57).

partition: GMRES iterations of the anisotropic reaction-diffusion problem
(equation (60) with a0 = 1e-6 and c0 in {1e-4, 1, 1e2, 1e3}) and of the
high-contrast Helmholtz problem (rho_D = 1e3 in the enclosure D) under the box,
horizontal-slab and vertical-slab partitions.

Every problem is real and factorized in FP64 (the workload generator's study
families); inputs are seeded and synthetic. The ID tolerance is --tol for every
run, or with --scale cond it follows the SIPG condition number, which grows as
p^4 / h^2: tol (n0 / n)^2 (p0 / p)^4 from the sweep's first point (n0, p0), so
that the perturbation the compression makes stays the same relative to it.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def run_one(P, hss):
    import torch
    t0 = time.perf_counter()
    h = hss.factor(P.op, P.tree, P.tol, prec=P.prec, seed=P.seed)
    torch.cuda.synchronize()
    t_factor = (time.perf_counter() - t0) * 1e3
    b = torch.from_numpy(np.ascontiguousarray(P.rhs[:, 0])).cuda()
    x, info = h.gmres(b, tol=P.gmres_tol, restart=P.restart, maxit=2000, raise_on_noconv=False)
    heap = h.query("node_heap").astype(int)
    ranks = h.query("ranks").astype(int)
    ls = h.query("l").astype(int)
    nbs = h.query("node_nb").astype(int)
    level = np.floor(np.log2(heap)).astype(int)
    cost = np.where(ranks > 0, ls * ranks * nbs * np.log(np.maximum(nbs, 2)), 0.0)
    top = int(np.nonzero(heap == 2)[0][0])
    out = {"name": P.name, "N": int(P.op.ndof), "n": int(P.op.n), "p": int(P.op.p), "iters": int(info[0]["iters"]),
           "true_relres": float(info[0]["true_relres"]), "factor_ms": round(t_factor, 2),
           "top_nb": int(nbs[top]), "top_k": int(ranks[top]), "top_l": int(ls[top]),
           "top_cost": float(cost[top]),
           "cost_per_level": {int(lv): float(cost[level == lv].sum()) for lv in np.unique(level)}}
    h.close()
    return out


def slope(xs, ys):
    """Least-squares slope of log y against log x."""
    lx, ly = np.log(np.asarray(xs, float)), np.log(np.asarray(ys, float))
    return float(np.polyfit(lx, ly, 1)[0]) if len(xs) > 1 else float("nan")


def study_hp(args, hss, configs):
    rows, fits = [], []
    for kind in args.kinds.split(","):
        for sweep, pts in (("h", [(int(n), args.p_h) for n in args.ns.split(",")]),
                           ("p", [(args.n_p, int(p)) for p in args.ps.split(",")])):
            runs = []
            n0, p0 = pts[0]
            for n, p in pts:
                tol = args.tol * ((n0 / n) ** 2 * (p0 / p) ** 4 if args.scale == "cond" else 1.0)
                r = run_one(configs.study(kind, n, p, tol=tol), hss)
                r.update({"kind": kind, "sweep": sweep, "tol": tol})
                print(json.dumps(r), flush=True)
                runs.append(r)
            rows += runs
            fit = {"kind": kind, "sweep": sweep, "scale": args.scale,
                   "k_vs_nb": slope([r["top_nb"] for r in runs], [max(r["top_k"], 1) for r in runs]),
                   "k_vs_log_nb": float(np.polyfit(np.log([r["top_nb"] for r in runs]),
                                                   [r["top_k"] for r in runs], 1)[0]) if len(runs) > 1 else None,
                   "top_cost_vs_N": slope([r["N"] for r in runs], [max(r["top_cost"], 1.0) for r in runs]),
                   "iters": [r["iters"] for r in runs]}
            print(json.dumps({"fit": fit}), flush=True)
            fits.append(fit)
    return {"runs": rows, "fits": fits}


def study_partition(args, hss, configs):
    rows = []
    cases = [("aniso", {"c0": c0}) for c0 in (1e-4, 1.0, 1e2, 1e3)] + [("contrast", {})]
    for kind, kw in cases:
        for scheme in ("boxes", "hslabs", "vslabs"):
            P = configs.study(kind, args.n, args.p, scheme=scheme, tol=args.tol, **kw)
            r = run_one(P, hss)
            r.update({"kind": kind, "scheme": scheme, "tol": args.tol, **kw})
            print(json.dumps(r), flush=True)
            rows.append(r)
    return {"runs": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("hp")
    a.add_argument("--kinds", default="poisson,cavity")
    a.add_argument("--ns", default="16,32,64,128")
    a.add_argument("--p-h", type=int, default=2)
    a.add_argument("--ps", default="1,2,3,4")
    a.add_argument("--n-p", type=int, default=32)
    a.add_argument("--tol", type=float, default=1e-3)
    a.add_argument("--scale", choices=("fixed", "cond"), default="fixed")
    a.add_argument("--json", default=None)
    b = sub.add_parser("partition")
    b.add_argument("--n", type=int, default=32)
    b.add_argument("--p", type=int, default=1)
    b.add_argument("--tol", type=float, default=1e-3)
    b.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    import torch  # device memory for the right-hand sides; initialised before the library
    if not torch.cuda.is_available():
        sys.exit("experiments.py needs a GPU")
    from paper_1508_07798_amd import hss
    from workloads import configs
    res = study_hp(args, hss, configs) if args.cmd == "hp" else study_partition(args, hss, configs)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
