"""Per-step kernel time of bench.py's timed steps from a rocprofv3 kernel trace.

    rocprofv3 --kernel-trace --output-format csv -d DIR -o run -- \\
        python3 bench.py --markers --steps K ...
    python profile_kernels.py --trace DIR --steps K --out profiles/X.md --title "..." --command "..."

bench.py --markers launches a spin kernel just before and just after its timed
steps; only the dispatches between the first two spin kernels are counted, so the
rank-model training, the warm-up and the FP64 comparison runs are left out. The
average duration per launch is what the bench's live roofline figure uses.
"""
import argparse
import collections
import csv
import glob
import os


def load(d):
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    return rows


def short(name):
    name = name.split("(")[0] if not name.startswith("void ") else name[5:].split("(")[0]
    return name.replace("hss::", "hss::")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--steps", type=int, required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    ap.add_argument("--top", type=int, default=30)
    a = ap.parse_args()
    rows = load(a.trace)
    marks = [i for i, r in enumerate(rows) if "spin_kernel" in r[2]]
    if len(marks) < 2:
        raise SystemExit("the trace holds no pair of marker kernels (run bench.py with --markers)")
    sel = rows[marks[0] + 1:marks[1]]
    agg = collections.defaultdict(lambda: [0, 0])
    for s, e, n in sel:
        agg[short(n)][0] += 1
        agg[short(n)][1] += e - s
    tot = sum(v[1] for v in agg.values())
    span = sel[-1][1] - sel[0][0] if sel else 0
    lines = [f"# {a.title}\n", "", "Command (from the repository root):", "", "```", a.command, "```", "",
             f"Dispatches between the two marker kernels, i.e. the {a.steps} timed steps of bench.py; "
             "times are per step, the average duration is per launch. The profiler adds roughly "
             "10 us between dispatches, so the span below is longer than the benchmark's step.", "",
             "| kernel | launches/step | ms/step | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, (cnt, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:a.top]:
        lines.append(f"| `{name}` | {cnt / a.steps:g} | {t / 1e6 / a.steps:.3f} | {t / cnt / 1e3:.2f} | "
                     f"{100.0 * t / tot:.2f} |")
    lines += ["", f"Total kernel time per step: {tot / 1e6 / a.steps:.2f} ms over "
              f"{len(sel) / a.steps:g} dispatches; first-to-last dispatch span per step "
              f"{span / 1e6 / a.steps:.2f} ms.", ""]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
