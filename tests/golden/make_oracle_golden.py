"""Write tests/golden/oracle_runs.json: GMRES iteration counts, ranks and
judge errors of the CPU oracle on the seeded workloads. Calls only oracle/
and workloads/ (the shared input generator).

    OPENBLAS_NUM_THREADS=1 python tests/golden/make_oracle_golden.py
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
         ("helmholtz_p2_64", None, None), ("varpoisson_p3_128", 16, None), ("varpoisson_p3_128", 32, None)]


def main():
    out = {}
    for name, n, p in CASES:
        P = configs.make(name, n=n, p=p)
        t0 = time.perf_counter()
        F = OracleFactor(P.op, P.tree, P.tol, seed=P.seed)
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = gmres(F.matvec, F.apply, P.rhs[:, 0], tol=P.gmres_tol, restart=P.restart)
        ts = time.perf_counter() - t0
        key = f"{name}@{P.op.n}"
        ranks = F.ranks()
        out[key] = dict(ndof=int(P.op.ndof), iters=int(res.iters), true_relres=float(res.true_relres),
                        max_err=float(F.max_err()), max_rank=int(max(ranks.values())),
                        mean_rank=float(np.mean(list(ranks.values()))),
                        ranks={str(s): int(k) for s, k in ranks.items()},
                        factor_s=tf, solve_s=ts)
        print(key, out[key]["iters"], out[key]["max_rank"], f"{tf:.1f}s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_runs.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
