"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2304_08232_amd.profsummary trace DIR [--cmd "..."]
      kernel time per (kernel, grid size) from a --kernel-trace run
      (rocpd SQLite database or kernel_trace.csv under DIR)
  python -m paper_2304_08232_amd.profsummary pmc DIR KERNEL_SUBSTR GRID [--cmd "..."]
      mean per-dispatch counter values (FETCH_SIZE / WRITE_SIZE, KiB) of the
      dispatches of one kernel at one grid size, and of the calibration copy
"""
import argparse
import csv
import glob
import os
import sqlite3
import sys
from collections import defaultdict


def _short(name):
    s = name.replace("void ", "").replace("mg::", "")
    return s.split("(")[0] if "(" in s and not s.startswith("(") else s


def load_trace(d):
    """[(name, grid, duration_ns)]"""
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    rows = []
    if dbs:
        c = sqlite3.connect(dbs[0])
        for name, grid, dur in c.execute("select name, grid_x, duration from kernels"):
            rows.append((name, int(grid), float(dur)))
        return rows
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0)))
            rows.append((r["Kernel_Name"], grid, float(r["End_Timestamp"]) - float(r["Start_Timestamp"])))
    return rows


def trace_summary(d, cmd, top=40):
    rows = load_trace(d)
    agg = defaultdict(lambda: [0, 0.0])
    for name, grid, dur in rows:
        a = agg[(_short(name), grid)]
        a[0] += 1
        a[1] += dur
    total = sum(v[1] for v in agg.values())
    out = [f"# rocprofv3 kernel trace summary", f"# command: {cmd}", f"# dispatches: {len(rows)}, "
           f"kernel time: {total / 1e6:.3f} ms", "",
           f"{'kernel':58s} {'grid':>9s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}"]
    for (name, grid), (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{name[:58]:58s} {grid:9d} {n:7d} {t / n / 1e3:9.3f} {t / 1e6:9.3f} {100 * t / total:6.2f}")
    return "\n".join(out)


def pmc_summary(d, kernel, grid, cmd):
    vals = defaultdict(lambda: defaultdict(list))
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    for f in files:
        for r in csv.DictReader(open(f)):
            g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)))
            key = "target" if (kernel in r["Kernel_Name"] and g == grid) else (
                "copy" if "copy" in r["Kernel_Name"].lower() or "elementwise" in r["Kernel_Name"] else None)
            if key:
                vals[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = [f"# rocprofv3 counter summary", f"# command: {cmd}", f"# kernel: {kernel} grid {grid}"]
    for key in ("target", "copy"):
        for cn, v in sorted(vals[key].items()):
            out.append(f"{key:6s} {cn:12s} dispatches {len(v):5d} mean {sum(v) / len(v):14.1f} KiB")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "pmc"])
    ap.add_argument("dir")
    ap.add_argument("kernel", nargs="?")
    ap.add_argument("grid", nargs="?", type=int)
    ap.add_argument("--cmd", default="")
    a = ap.parse_args()
    if a.mode == "trace":
        print(trace_summary(a.dir, a.cmd))
    else:
        print(pmc_summary(a.dir, a.kernel, a.grid, a.cmd))


if __name__ == "__main__":
    sys.exit(main())
