"""Matrix-core counters per kernel class from one rocprofv3 counter run.

    rocprofv3 --kernel-trace --pmc SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 \\
        SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE --output-format csv -d DIR -o run -- \\
        python3 bench.py --markers --steps 1 ...
    python profile_mfma.py --pmc DIR --classes NAME=REGEX ... --out profiles/X.md --command "..."

Only the dispatches between bench.py's two marker kernels are counted. For every
class (kernels whose name matches REGEX): the dispatch count, the counted
matrix-core flops (512 per MFMA MOP, F32 and F64 MOPs separately), the kernel
time from the trace of the same run, the flop rate that gives, and the ratio of
MFMA-busy cycles to the GPU-active cycles of the same dispatches (summed over
the dispatches).
"""
import argparse
import collections
import csv
import glob
import os
import re

COUNTERS = ["SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_VALU_MFMA_BUSY_CYCLES",
            "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"]


def load(d):
    """{dispatch id: (kernel name, {counter: value})} and {dispatch id: duration ns}."""
    disp = {}
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as f:
            for r in csv.DictReader(f):
                i = int(r["Dispatch_Id"])
                name, vals = disp.setdefault(i, (r["Kernel_Name"], {}))
                vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    dur = {}
    for fn in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(fn) as f:
            for r in csv.DictReader(f):
                dur[int(r["Dispatch_Id"])] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    if not disp:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return disp, dur


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pmc", required=True)
    ap.add_argument("--classes", nargs="+", required=True, help="NAME=REGEX")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    disp, dur = load(a.pmc)
    ids = sorted(disp)
    marks = [i for i in ids if "spin_kernel" in disp[i][0]]
    if len(marks) >= 2:
        ids = [i for i in ids if marks[0] < i < marks[1]]
    lines = [f"# {a.title}\n", "", "Command (from the repository root):", "", "```", a.command, "```", "",
             "Per class, over the dispatches between bench.py's marker kernels: counted matrix-core flops "
             "(512 per MFMA MOP), kernel time from the trace of the same run, their rate, and the ratio of "
             "MFMA-busy cycles to GPU-active cycles.", "",
             "| class | dispatches | MFMA flops F32 | MFMA flops F64 | kernel ms | counted TFLOP/s | "
             "MFMA busy / GPU active |", "|---|---:|---:|---:|---:|---:|---:|"]
    for spec in a.classes:
        cls, rx = spec.split("=", 1)
        sel = [i for i in ids if re.search(rx, disp[i][0])]
        if not sel:
            lines.append(f"| {cls} | 0 | | | | | |")
            continue
        tot = collections.defaultdict(float)
        for i in sel:
            for c, v in disp[i][1].items():
                tot[c] += v
        ns = sum(dur.get(i, 0) for i in sel)
        f32 = 512.0 * tot["SQ_INSTS_VALU_MFMA_MOPS_F32"]
        f64 = 512.0 * tot["SQ_INSTS_VALU_MFMA_MOPS_F64"]
        rate = (f32 + f64) / (ns * 1e-9) / 1e12 if ns else float("nan")
        busy = tot["SQ_VALU_MFMA_BUSY_CYCLES"] / tot["GRBM_GUI_ACTIVE"] if tot["GRBM_GUI_ACTIVE"] else float("nan")
        lines.append(f"| {cls} | {len(sel)} | {f32:.4g} | {f64:.4g} | {ns / 1e6:.2f} | {rate:.2f} | {busy:.3f} |")
    lines.append("")
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
