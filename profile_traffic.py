"""HBM traffic per launch of one kernel class from two rocprofv3 counter runs.

    python profile_traffic.py --fetch DIR --write DIR --cls gj_panel --regex gj_panel \
        --copy-mib 256 --sources FILE... --json OUT.json --summary OUT.md --command "..."

DIR holds the CSV output of `rocprofv3 --pmc FETCH_SIZE` (resp. WRITE_SIZE) of
`bench.py --copy-calib-mib N ...`. Both counters are in KiB per dispatch. Each
is scaled by what it reads for the plain device copy of N MiB that bench.py
runs first (the largest copy dispatch), so that the figure is in bytes moved.
The JSON records the sha256 of the kernel sources; bench.py uses the figure
only while those sources are unchanged.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.abspath(__file__))


def read_counter(d, counter):
    """(kernel, value) per dispatch in dispatch order. When the run holds bench.py's
    marker kernels (--markers), the dispatches between the first two markers are kept,
    plus the calibration copy, which bench.py runs before anything else."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter or "spin_kernel" in r.get("Kernel_Name", ""):
                    rows.append((int(r.get("Dispatch_Id", 0) or 0), r["Kernel_Name"],
                                 float(r["Counter_Value"]) if r.get("Counter_Name") == counter else None))
    rows.sort(key=lambda x: x[0])
    marks = [i for i, r in enumerate(rows) if "spin_kernel" in r[1]]
    copies = [(n, v) for _, n, v in rows if v is not None and ("copyBuffer" in n or "copy" in n.lower())]
    if len(marks) >= 2:
        rows = rows[marks[0] + 1:marks[1]]
    sel = [(n, v) for _, n, v in rows if v is not None and "spin_kernel" not in n]
    return copies + sel


def scaled(rows, regex, copy_mib):
    copies = [v for name, v in rows if "copyBuffer" in name or "copy" in name.lower()]  # calibration
    if not copies:
        raise SystemExit("no copy dispatch found for the calibration")
    ref = max(copies)
    scale = copy_mib * 1024.0 / ref  # true KiB per counted KiB
    sel = [v for name, v in rows if re.search(regex, name)]
    if not sel:
        raise SystemExit(f"no dispatch matches {regex}")
    return sum(sel) / len(sel) * scale * 1024.0, len(sel), ref, scale


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--cls", required=True)
    ap.add_argument("--regex", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--sources", nargs="+", required=True)
    ap.add_argument("--json", required=True)
    ap.add_argument("--summary", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--workload", default="helmholtz_p2_64")
    a = ap.parse_args()
    fb, nf, fref, fscale = scaled(read_counter(a.fetch, "FETCH_SIZE"), a.regex, a.copy_mib)
    wb, nw, wref, wscale = scaled(read_counter(a.write, "WRITE_SIZE"), a.regex, a.copy_mib)
    sources = {}
    for s in a.sources:
        with open(os.path.join(ROOT, s), "rb") as f:
            sources[s] = hashlib.sha256(f.read()).hexdigest()
    out = {"class": a.cls, "kernel_regex": a.regex, "bytes_per_launch": fb + wb,
           "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "dispatches": nf,
           "copy_mib": a.copy_mib, "copy_fetch_kib": fref, "copy_write_kib": wref,
           "fetch_scale": fscale, "write_scale": wscale, "sources": sources, "workload": a.workload}
    with open(a.json, "w") as f:
        json.dump(out, f, indent=1)
    with open(a.summary, "w") as f:
        f.write(f"# HBM traffic of `{a.cls}` kernels ({a.regex}), {a.workload}\n\n")
        f.write(f"Command:\n\n```\n{a.command}\n```\n\n")
        f.write(f"* dispatches counted: {nf} (FETCH_SIZE), {nw} (WRITE_SIZE)\n")
        f.write(f"* copy calibration: {a.copy_mib} MiB copy reads FETCH_SIZE {fref:.0f} KiB, "
                f"WRITE_SIZE {wref:.0f} KiB (scales {fscale:.4f}, {wscale:.4f})\n")
        f.write(f"* per launch: fetch {fb / 1e6:.4f} MB, write {wb / 1e6:.4f} MB, "
                f"total {(fb + wb) / 1e6:.4f} MB\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
