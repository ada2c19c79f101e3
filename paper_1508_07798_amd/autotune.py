"""Autotuner of the Gauss-Jordan elimination that inverts the box interiors.

For every scalar type and size class (boxes of at most 128 ... 4096 interior
rows) it times the elimination of a batch of random boxes of that size through
the library (hss_debug_gj) with every compiled compact panel shape that holds the
class's rows and a few second-level block widths, and writes the fastest to a JSON
file that the library reads (hss_tuning_load; by default tuning_gfx950.json beside
libhss.so). The built-in choice is kept unless another is faster by more than the
margin, so noise does not move the table.

    python -m paper_1508_07798_amd.autotune [--out FILE] [--reps N]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import hss

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning_gfx950.json")
CLASSES = (128, 256, 512, 1024, 2048, 4096)
TORCH_DT = {"float32": "float32", "float64": "float64", "complex64": "complex64", "complex128": "complex128"}


def _batch(scalar, rows, device, seed):
    """Boxes [A | B] with A = rows x rows (diagonal shifted so partial pivoting
    stays tame) and B = rows x rows/2, column-major (tensors shaped [cols, rows])."""
    import torch
    dt = getattr(torch, TORCH_DT[scalar])
    m = rows // 2
    nbox = int(max(2, min(256, (1 << 24) // (rows * (rows + m)))))
    g = torch.Generator(device="cpu").manual_seed(seed)
    mats = []
    for _ in range(nbox):
        a = torch.randn(rows + m, rows, generator=g, dtype=torch.float64)
        if dt.is_complex:
            a = torch.complex(a, torch.randn(rows + m, rows, generator=g, dtype=torch.float64))
        a[:rows].diagonal().add_(float(np.sqrt(rows)))
        mats.append(a.to(dt).to(device))
    return mats, [rows] * nbox, [m] * nbox


def _time(pristine, work, ns, ms, reps):
    import torch
    best = float("inf")
    for _ in range(reps):
        for w, p in zip(work, pristine):
            w.copy_(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if hss.debug_gj(work, ns, ms) != 0:
            raise RuntimeError("singular test box")
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best * 1e3


def tune(out=DEFAULT_OUT, scalars=("float32", "float64", "complex64", "complex128"), classes=CLASSES, reps=3,
         margin=0.03, device="cuda:0", log=print):
    import torch  # device memory for the test boxes; initialised before the library's first call
    assert torch.cuda.is_available(), "the autotuner needs a GPU"
    entries = []
    hss.tuning_clear()
    for si, scalar in enumerate(scalars):
        for rows in classes:
            cands = hss.tuning_candidates(scalar, rows)
            if not cands:
                continue  # taller than every compact shape: the tournament path, not tuned here
            pristine, ns, ms = _batch(scalar, rows, device, seed=1000 * si + rows)
            work = [p.clone() for p in pristine]
            blocks = [-1] if rows <= 128 else [-1, 0, 64, 128, 256]
            tried = []
            hss.tuning_set(scalar, rows)  # built-in rule
            t_def = _time(pristine, work, ns, ms, reps)
            tried.append({"nb": 0, "rpt": 0, "nt": 0, "block": -1, "ms": round(t_def, 4)})
            for nb, rpt, nt in cands:
                for blk in blocks:
                    hss.tuning_set(scalar, rows, nb, rpt, nt, blk)
                    t = _time(pristine, work, ns, ms, reps)
                    tried.append({"nb": nb, "rpt": rpt, "nt": nt, "block": blk, "ms": round(t, 4)})
            best = min(tried, key=lambda e: e["ms"])
            if best["ms"] > (1.0 - margin) * t_def:
                best = tried[0]
            hss.tuning_set(scalar, rows, best["nb"], best["rpt"], best["nt"], best["block"])
            entries.append({"scalar": scalar, "rows": rows, "nb": best["nb"], "rpt": best["rpt"], "nt": best["nt"],
                            "block": best["block"], "ms": best["ms"], "builtin_ms": round(t_def, 4),
                            "boxes": len(ns), "tried": tried})
            log(f"{scalar:10s} rows<={rows:5d}: built-in {t_def:8.3f} ms, chosen nb {best['nb']} rpt {best['rpt']} "
                f"nt {best['nt']} block {best['block']}: {best['ms']:8.3f} ms ({len(tried)} tried)")
            del pristine, work
    doc = {"arch": "gfx950", "tool": "paper_1508_07798_amd/autotune.py", "reps": reps, "margin": margin,
           "entries": entries}
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    return doc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    tune(a.out, reps=a.reps, log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
