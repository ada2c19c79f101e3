"""Write tests/golden/oracle_runs.json: GMRES iteration counts, ranks and
judge errors of the CPU oracle on the seeded workloads. Calls only oracle/
and workloads/ (the shared input generator).

    OPENBLAS_NUM_THREADS=1 python tests/golden/make_oracle_golden.py [key ...]

With keys, only those entries are recomputed and the others kept.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.factor import OracleFactor  # noqa: E402
from oracle.gmres import gmres  # noqa: E402
from workloads import configs  # noqa: E402

CASES = [("poisson_p1_16", None, None), ("helmholtz_p2_64", 16, None), ("helmholtz_p2_64", 32, None),
         ("helmholtz_p2_64", None, None), ("varpoisson_p3_128", 16, None), ("varpoisson_p3_128", 32, None),
         ("varpoisson_p3_128", None, None), ("helmholtz_p4_256", 16, None), ("helmholtz_p4_256", 32, None),
         ("helmholtz_p4_256", 64, None)]


def batch_subset():
    """Indices of the smallest, the largest and two middle-sized problems of the
    batched Helmholtz workload (by dof count, ties to the lower index)."""
    sizes = [P.op.ndof for P in configs.make_batch()]
    order = sorted(range(len(sizes)), key=lambda i: (sizes[i], i))
    return [order[0], order[len(order) // 3], order[(2 * len(order)) // 3], order[-1]]


def run(P, seed, cols):
    t0 = time.perf_counter()
    F = OracleFactor(P.op, P.tree, P.tol, seed=seed)
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = [gmres(F.matvec, F.apply, P.rhs[:, c], tol=P.gmres_tol, restart=P.restart) for c in cols]
    ts = time.perf_counter() - t0
    ranks = F.ranks()
    return dict(ndof=int(P.op.ndof), iters=int(res[0].iters), true_relres=float(res[0].true_relres),
                iters_rhs=[int(r.iters) for r in res], relres_rhs=[float(r.true_relres) for r in res],
                max_err=float(F.max_err()), max_rank=int(max(ranks.values())),
                mean_rank=float(np.mean(list(ranks.values()))),
                ranks={str(s): int(k) for s, k in ranks.items()}, seed=int(seed),
                factor_s=tf, solve_s=ts)


def main(only=None):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json")
    out = {}
    if only and os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for name, n, p in CASES:
        P = configs.make(name, n=n, p=p)
        key = f"{name}@{P.op.n}"
        if only and key not in only:
            continue
        out[key] = run(P, P.seed, [0])
        print(key, out[key]["iters"], out[key]["max_rank"], f"{out[key]['factor_s']:.1f}s", flush=True)
    # the batch: every problem of one batched factorization draws its test
    # matrices with the batch's seed (that of its first problem)
    batch = configs.make_batch()
    for i in batch_subset():
        P = batch[i]
        key = f"helmholtz_batch64#{i}@{P.op.n}"
        if only and key not in only:
            continue
        out[key] = run(P, batch[0].seed, list(range(P.rhs.shape[1])))
        print(key, out[key]["iters_rhs"], out[key]["max_rank"], f"{out[key]['factor_s']:.1f}s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(set(sys.argv[1:]) or None)
