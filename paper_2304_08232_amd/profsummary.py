"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2304_08232_amd.profsummary trace DIR [--cmd "..."] [--match REGEX]
      kernel time per (kernel, grid size) from a --kernel-trace run
      (rocpd SQLite database or kernel_trace.csv under DIR); --match keeps
      the kernels whose short name matches REGEX (e.g. the instantiations for
      16 right-hand sides)
  python -m paper_2304_08232_amd.profsummary pmc DIR KERNEL_SUBSTR GRID [--cmd "..."]
      mean per-dispatch counter values (FETCH_SIZE / WRITE_SIZE, KiB) of the
      dispatches of one kernel at one grid size, and of the calibration copy
  python -m paper_2304_08232_amd.profsummary traffic FETCH_DIR WRITE_DIR KERNEL_SUBSTR GRID
         [--copy-mib 512] [--json OUT] [--cmd "..."]
      HBM bytes per launch of one kernel from a FETCH_SIZE run and a
      WRITE_SIZE run, each counter scaled by what it reads for the largest
      device copy in the same run (a copy of --copy-mib MiB); --json writes
      the figure with the hash of the kernel sources it was taken on
  python -m paper_2304_08232_amd.profsummary traffic-all FETCH_DIR WRITE_DIR [--copy-mib 512] [--cmd "..."]
      the same for every (kernel, grid size) of the two runs, largest first
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
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


def trace_summary(d, cmd, top=40, match=None):
    rows = load_trace(d)
    if match:
        pat = re.compile(match)
        rows = [r for r in rows if pat.search(_short(r[0]))]
    agg = defaultdict(lambda: [0, 0.0])
    for name, grid, dur in rows:
        a = agg[(_short(name), grid)]
        a[0] += 1
        a[1] += dur
    total = sum(v[1] for v in agg.values())
    out = [f"# rocprofv3 kernel trace summary (grid = work-items of the dispatch)", f"# command: {cmd}",
           f"# dispatches: {len(rows)}, kernel time: {total / 1e6:.3f} ms", "",
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


def kernel_source_hash():
    """Hash of the kernel sources; a stored counter figure is valid only for it."""
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in ("kernels.hip", "wavefront.hip", "library.hip", "kernels.h", "mgpcg_internal.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_rows(d, counter):
    """[(kernel name, grid, value KiB)] of one counter over a --pmc run."""
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)))
                out.append((r["Kernel_Name"], g, float(r["Counter_Value"])))
    return out


def traffic(fetch_dir, write_dir, kernel, grid, copy_mib=512):
    res = {"kernel": kernel, "grid": grid, "copy_mib": copy_mib}
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = _counter_rows(d, counter)
        tgt = [v for n, g, v in rows if kernel in n and g == grid]
        copies = [v for n, g, v in rows if "copyBuffer" in n]
        if not tgt or not copies:
            raise SystemExit(f"{counter}: no dispatches of {kernel} at grid {grid} or no copy in {d}")
        ref = max(copies)
        res[f"{tag}_kib_mean"] = sum(tgt) / len(tgt)
        res[f"{tag}_dispatches"] = len(tgt)
        res[f"copy_{tag}_kib"] = ref
        res[f"{tag}_factor"] = copy_mib * 1024.0 / ref
    res["hbm_bytes_per_launch"] = int(round(1024.0 * (res["fetch_kib_mean"] * res["fetch_factor"] +
                                                      res["write_kib_mean"] * res["write_factor"])))
    res["kernel_source_hash"] = kernel_source_hash()
    return res


def traffic_all(fetch_dir, write_dir, copy_mib=512):
    """{(kernel, grid): (dispatches, fetch bytes, write bytes)} per dispatch, scaled."""
    acc = defaultdict(lambda: [0, 0.0, 0.0])
    for col, d, counter in ((1, fetch_dir, "FETCH_SIZE"), (2, write_dir, "WRITE_SIZE")):
        rows = _counter_rows(d, counter)
        copies = [v for n, g, v in rows if "copyBuffer" in n]
        if not copies:
            raise SystemExit(f"{counter}: no copy in {d}")
        factor = copy_mib * 1024.0 / max(copies)
        for n, g, v in rows:
            if "copyBuffer" in n:
                continue
            a = acc[(_short(n), g)]
            if col == 1:
                a[0] += 1
            a[col] += 1024.0 * v * factor
    return {k: (a[0], a[1] / max(a[0], 1), a[2] / max(a[0], 1)) for k, a in acc.items()}


def traffic_all_summary(t, cmd):
    out = ["# rocprofv3 counter summary: HBM bytes per dispatch of every kernel",
           "# (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a device copy of known size)",
           f"# commands: {cmd}", "",
           f"{'kernel':58s} {'grid':>9s} {'calls':>6s} {'read_MB':>9s} {'write_MB':>9s} {'total_MB':>9s}"]
    for (name, grid), (n, f, w) in sorted(t.items(), key=lambda kv: -(kv[1][1] + kv[1][2]) * kv[1][0]):
        out.append(f"{name[:58]:58s} {grid:9d} {n:6d} {f / 1e6:9.2f} {w / 1e6:9.2f} {(f + w) / 1e6:9.2f}")
    return "\n".join(out)


def traffic_summary(t, cmd):
    return "\n".join([
        "# rocprofv3 counter summary: HBM traffic of one kernel",
        f"# commands: {cmd}",
        f"# kernel: {t['kernel']} grid {t['grid']} (kernel sources {t['kernel_source_hash']})",
        f"FETCH_SIZE  mean {t['fetch_kib_mean']:12.1f} KiB over {t['fetch_dispatches']} dispatches; "
        f"{t['copy_mib']} MiB copy reads {t['copy_fetch_kib']:.1f} KiB -> x{t['fetch_factor']:.3f}",
        f"WRITE_SIZE  mean {t['write_kib_mean']:12.1f} KiB over {t['write_dispatches']} dispatches; "
        f"{t['copy_mib']} MiB copy reads {t['copy_write_kib']:.1f} KiB -> x{t['write_factor']:.3f}",
        f"HBM bytes per launch (scaled): {t['hbm_bytes_per_launch']} "
        f"({t['hbm_bytes_per_launch'] / 1e6:.2f} MB)"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "pmc", "traffic", "traffic-all"])
    ap.add_argument("dir")
    ap.add_argument("args", nargs="*")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--json", default=None)
    ap.add_argument("--match", default=None)
    a = ap.parse_args()
    if a.mode == "trace":
        print(trace_summary(a.dir, a.cmd, match=a.match))
    elif a.mode == "pmc":
        print(pmc_summary(a.dir, a.args[0], int(a.args[1]), a.cmd))
    elif a.mode == "traffic-all":
        print(traffic_all_summary(traffic_all(a.dir, a.args[0], a.copy_mib), a.cmd))
    else:
        t = traffic(a.dir, a.args[0], a.args[1], int(a.args[2]), a.copy_mib)
        t["command"] = a.cmd
        print(traffic_summary(t, a.cmd))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(t, f, indent=1)
                f.write("\n")


if __name__ == "__main__":
    sys.exit(main())
