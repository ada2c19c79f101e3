"""Benchmark: setup (hss_factor) + GMRES solve to 1e-8 on one MI355X.

A step is the whole hot path on one synthetic input: hss_factor of the measured
workload followed by gmres_solve in FP64 (complex128) to a true relative
residual of 1e-8. The operator values and the right-hand sides are resident in
HBM before the timed region. The same steps are timed in the plain FP64 form
for the mixed-versus-FP64 comparison, the mixed form is timed once more without
the rank model (plain adaptive ID), and the CPU oracle is timed on the host on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CLASSES = ["gather", "gj_panel", "gj_rows", "gj_update", "gj_perm", "schur_gemm", "symm", "omega",
           "sample_gemm", "sample", "id", "utall", "expand", "judge", "root", "apply", "spmv", "gmres",
           "gj_panel_wide", "gj_rows_wide", "gj_update_wide"]
# MI355X peaks: dense MFMA FP32 / FP64, vector FP32 / FP64, HBM3E
PEAK = {"mfma_fp32": 157.3, "mfma_fp64": 78.6, "mfma_bf16": 2500.0, "alu_fp32": 157.3, "alu_fp64": 78.6,
        "hbm": 8000.0}
# bound of each kernel class and whether its algorithmic work is counted in flops or bytes
BOUND = {"gather": "hbm", "gj_panel": "alu", "gj_rows": "hbm", "gj_update": "mfma", "schur_gemm": "mfma",
         "symm": "hbm", "omega": "hbm", "sample_gemm": "mfma", "sample": "mfma", "id": "alu", "utall": "alu",
         "expand": "mfma", "judge": "hbm", "apply": "hbm", "spmv": "hbm", "root": "hbm", "gj_perm": "hbm",
         "gj_panel_wide": "alu", "gj_rows_wide": "hbm", "gj_update_wide": "mfma"}
# the *_wide classes: Gauss-Jordan work that a single-precision factorization does in
# double precision (complex64 boxes above 2048 interior rows, and the root)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "roofline_traffic.json")
# measured workloads: the mixed form's precision and the arithmetic type it computes in
WORKLOADS = {
    "helmholtz_p4_256": {"mixed": "fp32", "dtype": "c64", "model": "configs123",
                         "desc": "helmholtz_p4_256: impedance Helmholtz, SIPG p=4, 256x256 elements, 1638400 "
                                 "dofs, 10 dofs/wavelength, ID tol 1e-4, GMRES(30) to 1e-8"},
    "helmholtz_p2_64": {"mixed": "fp32", "dtype": "c64",
                        "desc": "helmholtz_p2_64: impedance Helmholtz, SIPG p=2, 64x64 elements, 36864 dofs, "
                                "8 dofs/wavelength, ID tol 1e-4, GMRES(30) to 1e-8"},
    "varpoisson_p3_128": {"mixed": "bf16", "dtype": "f32 (bf16 Schur products)",
                          "desc": "varpoisson_p3_128: -div(a grad u), a = exp(GRF l=0.1, var 1), SIPG p=3, "
                                  "128x128 elements, 262144 dofs, ID tol 1e-5, GMRES(30) to 1e-8"},
    "helmholtz_batch64": {"mixed": "fp32", "dtype": "c64", "family": "helmholtz_p2_64",
                          "desc": "helmholtz_batch64: 64 impedance Helmholtz problems, grids U{32..96}, SIPG p=2, "
                                  "6-10 dofs/wavelength, 4 point sources each, one batched factorization and "
                                  "solve, ID tol 1e-4, GMRES(30) to 1e-8"},
}
DEFAULT_WORKLOAD = "helmholtz_p4_256"


def class_table(h, steps=1):
    """Per-class time, launches and algorithmic work from a handle's HIP-event profile."""
    out = {}
    for c in CLASSES:
        ms = float(h.query(f"prof.{c}.ms")[0]) / steps
        n = float(h.query(f"prof.{c}.launches")[0]) / steps
        if n == 0:
            continue
        fl = float(h.query(f"prof.{c}.flops")[0]) / steps
        by = float(h.query(f"prof.{c}.bytes")[0]) / steps
        out[c] = {"ms": ms, "launches": n, "flops": fl, "bytes": by}
    return out


def roofline_entry(cls, rec, fp64, bf16_schur=False):
    bound = BOUND.get(cls, "alu")
    fp64 = fp64 or cls.endswith("_wide")
    if bf16_schur and cls == "schur_gemm":  # BF16 matrix cores (algorithmic flops, dense BF16 peak)
        achieved = rec["flops"] / (rec["ms"] * 1e-3) / 1e12 if rec["flops"] > 0 else None
        return {"bound": "mfma", "achieved": None if achieved is None else round(achieved, 4),
                "peak": PEAK["mfma_bf16"], "unit": "TFLOP/s",
                "frac": None if achieved is None else round(achieved / PEAK["mfma_bf16"], 5),
                "avg_launch_ms": round(rec["ms"] / rec["launches"], 5),
                "work_per_launch": rec["flops"] / rec["launches"], "ms_per_step": round(rec["ms"], 4)}
    if bound == "hbm":
        peak, unit, work = PEAK["hbm"], "GB/s", rec["bytes"]
        achieved = work / (rec["ms"] * 1e-3) / 1e9 if work > 0 else None
    else:
        peak = PEAK[f"{bound}_{'fp64' if fp64 else 'fp32'}"]
        unit, work = "TFLOP/s", rec["flops"]
        achieved = work / (rec["ms"] * 1e-3) / 1e12 if work > 0 else None
    return {"bound": bound, "achieved": None if achieved is None else round(achieved, 4), "peak": peak,
            "unit": unit, "frac": None if achieved is None else round(achieved / peak, 5),
            "avg_launch_ms": round(rec["ms"] / rec["launches"], 5),
            "work_per_launch": work / rec["launches"], "ms_per_step": round(rec["ms"], 4)}


def sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(cls, workload):
    """HBM bytes per launch of `cls` from the committed counter summary, or None when
    the summary covers another class or workload, or its kernel sources have changed
    since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("class") != cls or t.get("workload") != workload:
        return None
    for rel, digest in t.get("sources", {}).items():
        if sha256(os.path.join(ROOT, rel)) != digest:
            return None
    return t.get("bytes_per_launch")


def blas_info():
    """BLAS library and thread count numpy uses (threadpoolctl), or None."""
    try:
        from threadpoolctl import threadpool_info
        return [{k: d.get(k) for k in ("internal_api", "version", "num_threads")} for d in threadpool_info()
                if d.get("user_api") == "blas"]
    except Exception:
        return None


def structural_flops(P):
    """LU + triangular solves + Schur products of every box and the root's LU (real
    flops, x4 complex) from the planner's sets: the part of the method's work fixed by
    the structure alone (no GPU needed)."""
    from paper_1508_07798_amd import hss
    pl = hss.Plan(P.op, P.tree)
    cx = 4.0 if P.op.is_complex else 1.0
    f = 0.0
    for depth in range(1, 40):
        found = False
        for s in range(2 ** depth, 2 ** (depth + 1)):
            try:
                ni = float(pl.query("idof", s).size)
                nb = float(pl.query("bdof", s).size)
            except Exception:
                continue
            found = True
            f += cx * ((2.0 / 3.0) * ni ** 3 + 2.0 * ni * ni * nb + 2.0 * nb * nb * ni)
        if not found and depth > 1:
            break
    nr = float(pl.query("root").size)
    f += cx * (2.0 / 3.0) * nr ** 3
    pl.close()
    return f


def cpu_baseline(probs, budget_s=20.0):
    """The oracle as it stands on the host's cores (multithreaded BLAS): factor and
    GMRES (every right-hand side) of the workload's problems in order, or, for a
    workload beyond about budget_s of host time, of a smaller seeded problem of the
    same family; the time is scaled to the whole workload by the ratio of the
    structural flops (LU, triangular solves, Schur products, root LU)."""
    from oracle.factor import OracleFactor
    from oracle.gmres import gmres as ogmres
    full = sum(structural_flops(P) for P in probs)
    t_all = 0.0
    done_flops = 0.0
    iters = []
    names = []
    for P in probs:
        t0 = time.perf_counter()
        F = OracleFactor(P.op, P.tree, P.tol, seed=P.seed)
        for c in range(P.rhs.shape[1] if len(probs) > 1 else 1):
            iters.append(ogmres(F.matvec, F.apply, P.rhs[:, c], tol=P.gmres_tol, restart=P.restart).iters)
        t_all += time.perf_counter() - t0
        done_flops += structural_flops(P)
        names.append(f"{P.name}@{P.op.n}")
        if t_all >= budget_s:
            break
    return {"seconds": t_all, "sample": names, "scale": full / done_flops, "iters": iters}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=None, help="0 skips the FP64 form")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--roofline-class", default=None,
                    help="kernel class for the roofline object (default: the dominant one)")
    ap.add_argument("--profile-all", action="store_true", help="print the time of every kernel class")
    ap.add_argument("--no-model", action="store_true", help="plain adaptive ID (no rank model)")
    ap.add_argument("--markers", action="store_true",
                    help="spin kernels around the timed steps, to cut a kernel trace to them")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS),
                    help="measured workload (default: the largest configuration, p=4 Helmholtz on 256x256)")
    ap.add_argument("--mixed", default=None, choices=("fp32", "bf16"),
                    help="precision of the mixed form's Schur products (default: the workload's)")
    ap.add_argument("--oracle-sample-n", type=int, default=16,
                    help="grid of the smaller same-family problem the oracle is timed on when the "
                         "workload itself is too large for the host")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the path would shard by subtree, one GPU per subtree).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1508_07798_amd import hss
    from workloads import configs

    W = WORKLOADS[args.workload]
    MIX = args.mixed or W["mixed"]
    def note(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    note(f"building {args.workload}")
    probs = configs.make_batch() if args.workload == "helmholtz_batch64" else [configs.make(args.workload)]
    P = probs[0]
    note(f"{len(probs)} problem(s), {sum(q.op.ndof for q in probs)} dofs")
    dev = torch.device("cuda:0")
    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    vals = [torch.from_numpy(q.op.vals).to(dev) for q in probs]
    batched = len(probs) > 1
    # a single problem solves its first rhs; the batch solves every rhs of every problem
    b = torch.from_numpy(np.ascontiguousarray(np.concatenate([q.rhs if batched else q.rhs[:, :1] for q in probs],
                                                             axis=0))).to(dev)
    # kappa * h is one feature per handle: the batch takes the mean
    kh = float(np.mean([q.kappa / q.op.n if q.kappa else 0.0 for q in probs]))
    tol = probs[0].tol

    # the rank model is trained once, before any timing, on smaller seeded problems
    from paper_1508_07798_amd import rank_model
    model = None
    minfo = None
    if not args.no_model:
        note("training the rank model")
        model, minfo = rank_model.fit_default(family=W.get("model", W.get("family", args.workload)), prec=MIX)
        minfo["trained_on"] = ("the Poisson p=1, Helmholtz p=2 and variable-coefficient Poisson p=3 runs"
                               if W.get("model") == "configs123" else
                               f"smaller seeded problems of the {W.get('family', args.workload)} family")

    def step(prec, profile, use_model=True):
        h = hss.factor_batched([q.op for q in probs], [q.tree for q in probs], tol, prec=prec, seed=P.seed,
                               vals_dev=vals, profile=profile, kappa_h=kh,
                               rank_model=model if use_model else None)
        x, info = h.gmres(b, tol=P.gmres_tol, restart=P.restart, nprob=len(probs))
        return h, x, info

    def stats(h, info):
        """What the report needs from a handle (queried before it is closed)."""
        return {"iters": max(i["iters"] for i in info), "relres": max(i["true_relres"] for i in info),
                "table": class_table(h), "flops_factor": float(h.query("flops_factor")[0]),
                "flops_parts": h.query("flops_factor_parts"), "flops_gj": float(h.query("flops_gj")[0]),
                "ranks": np.asarray(h.query("ranks")), "l_init": np.asarray(h.query("l_init")),
                "t_factor": float(h.query("time_factor_ms")[0]), "t_wait": float(h.query("host_wait_ms")[0]),
                "phases": h.query("phase_ms"), "max_rank": int(h.query("ranks").max()),
                "attempts": np.asarray(h.query("attempts")), "retries": float(h.query("retries")[0])}

    def timed(prec, steps, warmup, profile, use_model=True, markers=False):
        """Each step factors, solves, reads its statistics and frees the handle, so
        that the device memory of one step is reused by the next. HIP events (about
        10 us of device time per record) time the profiled class in the last step only.
        markers: a spin kernel on each side of the timed steps (outside the timed
        region), so that a kernel trace can be cut to exactly these steps."""
        for _ in range(warmup):
            h, _, _ = step(prec, 0, use_model)
            h.close()
        if markers:
            torch.cuda._sleep(1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        diag = 0.0
        for i in range(steps):
            h, x, info = step(prec, profile if i == steps - 1 else 0, use_model)
            # the solve has returned (its statistics are on the host), so the device is
            # idle: reading the handle's diagnostics is left out of the step time
            td = time.perf_counter()
            out.append(stats(h, info))
            diag += time.perf_counter() - td
            h.close()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0 - diag) * 1e3 / steps
        out[-1]["diag_ms"] = diag * 1e3 / steps
        if markers:
            torch.cuda._sleep(1000)
            torch.cuda.synchronize()
        return ms, out

    # one plain step loads every kernel's code and builds the first apply graph, then one
    # profiled warm-up step names the dominant kernel class (wrapper class gmres excluded)
    h, _, _ = step(MIX, 0)
    h.close()
    h, _, _ = step(MIX, 1)
    warm = class_table(h)
    h.close()
    dom = args.roofline_class or max((c for c in warm if c != "gmres"), key=lambda c: warm[c]["ms"])
    cls_bit = 1 << (CLASSES.index(dom) + 1)
    # timed steps: HIP events only around the dominant class's launches
    note(f"timing {args.steps} steps ({MIX})")
    ms, runs = timed(MIX, args.steps, args.warmup, cls_bit, markers=args.markers)
    iters = [r["iters"] for r in runs]
    relres = max(r["relres"] for r in runs)
    tot = runs[-1]["table"][dom]
    roof = roofline_entry(dom, tot, fp64=False, bf16_schur=MIX == "bf16")
    roof["kernel"] = dom
    roof["traffic"] = measured_traffic(dom, args.workload)
    flops_factor = runs[-1]["flops_factor"]
    t_factor = float(np.mean([r["t_factor"] for r in runs]))
    t_wait = float(np.mean([r["t_wait"] for r in runs]))
    phases = np.mean([r["phases"] for r in runs], axis=0)
    max_rank = runs[-1]["max_rank"]
    # per-class table from one more profiled step
    h, _, _ = step(MIX, 1)
    table = class_table(h)
    h.close()
    classes = {c: roofline_entry(c, rec, fp64=False, bf16_schur=MIX == "bf16") for c, rec in table.items()
               if c != "gmres"}

    # the same mixed form without the rank model (plain adaptive ID)
    plain = None
    if model is not None:
        note("timing the plain adaptive form")
        ms_plain, runs_plain = timed(MIX, max(1, min(3, args.steps // 2)), 1, 0, use_model=False)
        att_m = runs[-1]["attempts"]
        att_p = runs_plain[-1]["attempts"]
        plain = {"ms_per_step": round(ms_plain, 3), "gmres_iters": runs_plain[-1]["iters"],
                 "factor_ms": round(float(np.mean([r["t_factor"] for r in runs_plain])), 3),
                 "compress_attempts": int(att_p.sum()),
                 "boxes_retried_frac": round(float(np.mean(att_p[att_p > 0] > 1)), 4)}
        # a box is mispredicted when its rank exceeds what the predicted sample can
        # certify (k > l_init - p_os): the judge then grows its sample
        k_m, l0_m = runs[-1]["ranks"], runs[-1]["l_init"]
        comp = k_m > 0
        minfo.update({"compress_attempts": int(att_m.sum()),
                      "boxes_retried_frac": round(float(np.mean(att_m[att_m > 0] > 1)), 4),
                      "mispredicted_rank_frac": round(float(np.mean(k_m[comp] > l0_m[comp] - 10)), 4),
                      "mean_sample_over_rank": round(float(np.mean(l0_m[comp] / (k_m[comp] + 10))), 3),
                      "time_saved_ms": round(ms_plain - ms, 3),
                      "speedup_vs_plain": round(ms_plain / ms, 3)})

    fsteps = args.fp64_steps if args.fp64_steps is not None else max(1, min(3, args.steps // 2))
    ms64 = iters64 = t_factor64 = None
    if fsteps > 0:
        note("timing the FP64 form")
        ms64, runs64 = timed("fp64", fsteps, 1, 0)
        iters64 = runs64[-1]["iters"]
        t_factor64 = float(np.mean([r["t_factor"] for r in runs64]))

    if args.profile_all:
        for c in sorted(classes, key=lambda c: -classes[c]["ms_per_step"]):
            e = classes[c]
            print(f"  {c:12s} {e['ms_per_step']:8.3f} ms  {e['bound']:4s} achieved {e['achieved']} {e['unit']}"
                  f"  frac {e['frac']}", file=sys.stderr)

    cpu = None
    if not args.no_cpu:
        note("timing the oracle on the host")
        if args.workload == "helmholtz_p4_256":
            # the oracle on the full 1.6M-dof problem takes hours: a smaller seeded problem of
            # the same family (same p, dofs per wavelength and tol) is timed and scaled
            sample_probs = [configs.make(args.workload, n=args.oracle_sample_n)]
        else:
            sample_probs = probs
        cb = cpu_baseline(sample_probs)
        scale = cb["scale"] * (sum(structural_flops(q) for q in probs) /
                               sum(structural_flops(q) for q in sample_probs))
        cpu = {"value": round(cb["seconds"] * 1e3 * scale, 1), "unit": "ms", "cores": os.cpu_count(),
               "kind": "oracle", "blas": blas_info(),
               "sample": (f"oracle factor + GMRES of {', '.join(cb['sample'])} "
                          f"({len(cb['iters'])} solves) on the host's cores through multithreaded BLAS, "
                          f"{cb['seconds']:.1f} s measured, scaled by x{scale:.4g}, the ratio of the "
                          f"workload's structural flops (LU, triangular solves, Schur products, root LU) "
                          f"to the sample's"),
               "measured_s": round(cb["seconds"], 3), "oracle_gmres_iters": cb["iters"]}

    out = {
        "metric": "setup+GMRES time to 1e-8 resid, mixed vs FP64; factor TFLOP/s; GMRES iters",
        "value": round(ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": W["dtype"] if MIX == W["mixed"] else f"{W['dtype']} ({MIX} Schur products)",
        "data": "synthetic",
        "config": {"workload": W["desc"], "global_batch": 1, "parallelism": "single GPU"},
        "fp64_ms_per_step": None if ms64 is None else round(ms64, 3),
        "speedup_vs_fp64": None if ms64 is None else round(ms64 / ms, 3),
        "diagnostics_ms_excluded": round(runs[-1]["diag_ms"], 3),
        "factor_ms": round(t_factor, 3),
        "factor_host_wait_ms": round(t_wait, 3),
        "factor_phase_ms": dict(zip(["upload", "features", "gather", "gauss_jordan", "schur", "compression",
                                     "root", "apply_setup"], [round(float(v), 3) for v in phases])),
        "factor_ms_fp64": None if t_factor64 is None else round(t_factor64, 3),
        "factor_tflops": round(flops_factor / (t_factor * 1e-3) / 1e12, 4),
        "factor_flops": flops_factor,
        "factor_flops_parts": dict(zip(["lu", "trsm", "schur_gemm", "root_lu", "sampling", "cpqr"],
                                       [float(v) for v in runs[-1]["flops_parts"]])),
        "gj_form_flops": runs[-1]["flops_gj"],
        "gj_form_tflops": round(runs[-1]["flops_gj"] / (t_factor * 1e-3) / 1e12, 4),
        "gmres_iters": iters[-1],
        "gmres_iters_fp64": iters64,
        "true_relres": relres,
        "max_rank": max_rank,
        "rank_model": minfo,
        "plain_adaptive": plain,
        "roofline": roof,
        "kernel_classes": classes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
