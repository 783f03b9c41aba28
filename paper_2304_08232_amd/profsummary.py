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
  python -m paper_2304_08232_amd.profsummary breakdown DIR --dims NX NY NZ [--levels 4] [--cmd "..."]
         [--json OUT]
      where one CG iteration's time goes (the analogue of the per-level,
      per-operation breakdown of the paper's Sec. V-C): the dispatches of the
      solves in a --kernel-trace run (from the first k_init_residual on),
      grouped by multigrid level and phase, per iteration, with the nominal
      bytes of each level and the trace span per iteration
  python -m paper_2304_08232_amd.profsummary iteration-traffic FETCH_DIR WRITE_DIR [--copy-mib 512]
         [--json OUT] [--cmd "..."]
      HBM bytes of one CG iteration: the counter values of the dispatches
      after the first k_init_residual of each run, scaled as in `traffic`,
      summed and divided by the number of iterations (k_spmv_pq dispatches)
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


# ---------------------------------------------------- per-level breakdown

def load_trace_timed(d):
    """[(start_ns, end_ns, name, grid)] of a --kernel-trace run (CSV or rocpd)."""
    rows = []
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if dbs:
        c = sqlite3.connect(dbs[0])
        for st, en, name, grid in c.execute("select start, end, name, grid_x from kernels"):
            rows.append((float(st), float(en), name, int(grid)))
    else:
        for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0)))
                rows.append((float(r["Start_Timestamp"]), float(r["End_Timestamp"]), r["Kernel_Name"], grid))
    rows.sort()
    return rows


def _template_args(short):
    m = re.search(r"<(.*)>", short)
    return [a.strip() for a in m.group(1).split(",")] if m else []


def _level_grids(dims, levels):
    """grid size (work-items) -> level, for the per-colour passes, the
    two-colour zero-start launch and the unfused transfers"""
    from .perfmodel import level_sizes
    sz = level_sizes(dims, levels)
    up = lambda v, b: (v + b - 1) // b * b  # noqa: E731
    passes, zs01, transfers = {}, {}, {}
    for l, (n, _) in enumerate(sz):
        c = n // 8
        for b in (64, 256):
            passes.setdefault(up(c, b), l)
            zs01.setdefault(up(2 * c, b), l)
        if l + 1 < levels:
            transfers.setdefault(up(sz[l + 1][0], 256), l)
    return passes, zs01, transfers


PHASES = ["smoother", "smoother + restriction", "smoother + refinement", "restriction", "refinement",
          "coarsest level (one workgroup)", "coarse levels (persistent)", "zero fill", "FP32 casts",
          "CG SpMV + <p,q>", "CG vector updates and dots", "CG reductions (finalize)"]


def classify(short, grid, maps, levels):
    """(level or 'CG', phase) of one dispatch of an iteration, or None."""
    passes, zs01, transfers = maps
    base = short.split("<")[0]
    args = _template_args(short)
    if base == "k_pass":
        mode = int(args[4]) if len(args) > 4 else 0
        ph = {0: "smoother", 1: "smoother + restriction", 2: "smoother + refinement"}[mode]
        return passes.get(grid, "?"), ph
    if base == "k_pass_zs01":
        return zs01.get(grid, "?"), "smoother"
    if base == "k_coarse_tail":
        return levels - 1, "coarsest level (one workgroup)"
    if base == "k_coarse_vcycle":
        return "1+", "coarse levels (persistent)"
    if base == "k_restrict":
        return transfers.get(grid, "?"), "restriction"
    if base == "k_prolong":
        return transfers.get(grid, "?"), "refinement"
    if base in ("k_cast_d2f", "k_cast_f2d"):
        return 0, "FP32 casts"
    if base == "k_fill":
        return "?", "zero fill"
    if base == "k_spmv_pq":
        return "CG", "CG SpMV + <p,q>"
    if base in ("k_update_p", "k_update_r", "k_flush_x", "k_dot_rz"):
        return "CG", "CG vector updates and dots"
    if base in ("k_finalize", "k_fold"):
        return "CG", "CG reductions (finalize)"
    return None


def breakdown(d, dims, levels=4):
    from .perfmodel import level_sizes
    rows = load_trace_timed(d)
    first = next((k for k, r in enumerate(rows) if _short(r[2]).startswith("k_init_residual")), None)
    if first is None:
        raise SystemExit(f"no k_init_residual dispatch in {d}")
    # the solves' dispatches; the initial residual's reduction and finalize
    # (once per solve) are set-up, not iteration work
    sol, prev = [], ""
    for r in rows[first:]:
        sh = _short(r[2])
        if not sh.startswith("k_"):
            continue
        if prev.startswith("k_init_residual") and sh.startswith(("k_finalize", "k_fold")):
            sol.append((r[0], r[1], "setup:" + r[2], r[3]))
            continue
        sol.append(r)
        prev = sh
    iters = sum(1 for r in sol if _short(r[2]).startswith("k_spmv_pq"))
    if iters == 0:
        raise SystemExit("no CG iteration in the trace")
    maps = _level_grids(dims, levels)
    agg = defaultdict(lambda: [0, 0.0])
    setup_ns = 0.0
    for st, en, name, grid in sol:
        short = _short(name)
        c = None if name.startswith("setup:") else classify(short, grid, maps, levels)
        if c is None:  # per-solve set-up (initial residual, fills of the CG state)
            setup_ns += en - st
            continue
        a = agg[c]
        a[0] += 1
        a[1] += en - st
    last_end = max(r[1] for r in sol)
    span = (last_end - sol[0][0]) / iters
    kern = sum(a[1] for a in agg.values()) / iters
    # nominal bytes (perfmodel's terms) by level and for the CG part
    sz = level_sizes(dims, levels)
    nominal = {}
    for l, (n, nnz) in enumerate(sz):
        b = (2 if l == levels - 1 else 4) * (12 * nnz + 24 * n) + 8 * n
        if l < levels - 1:
            b += 12 * nnz + 16 * n + 2 * 24 * sz[l + 1][0]
        nominal[l] = b
    n0, nnz0 = sz[0]
    nominal["CG"] = 12 * nnz0 + 16 * n0 + 40 * n0 + 72 * n0
    return {"dims": list(dims), "levels": levels, "iterations": iters,
            "span_us_per_iteration": span / 1e3, "kernel_us_per_iteration": kern / 1e3,
            "setup_us_per_iteration": setup_ns / iters / 1e3,
            "groups": [{"level": str(k[0]), "phase": k[1], "launches": a[0] / iters, "us": a[1] / iters / 1e3}
                       for k, a in agg.items()],
            "nominal_bytes": {str(k): v for k, v in nominal.items()}}


def breakdown_summary(b, cmd, wall_us=None):
    """wall_us: the iteration time measured without the profiler; each
    group's share of the traced kernel time is also shown scaled to it."""
    key = lambda g: (g["level"] == "CG", g["level"], PHASES.index(g["phase"]) if g["phase"] in PHASES else 99)  # noqa: E731
    groups = sorted(b["groups"], key=key)
    kern = b["kernel_us_per_iteration"]
    scale = (wall_us / kern) if wall_us else None
    sc_h = f" {'us_scaled':>9s}" if scale else ""
    out = ["# where one MG-PCG iteration's time goes, by multigrid level and phase",
           f"# command: {cmd}",
           f"# grid {'x'.join(map(str, b['dims']))}, {b['levels']} levels, {b['iterations']} iterations traced",
           f"# kernel time per iteration under the tracer {kern:.1f} us; trace span per iteration "
           f"{b['span_us_per_iteration']:.1f} us (launch gaps, per-solve set-up, tracer overhead)"]
    if scale:
        out.append(f"# us_scaled: each group's share of the traced kernel time times the iteration time "
                   f"measured without the profiler, {wall_us:.1f} us")
    out += ["", f"{'level':6s} {'phase':34s} {'launches':>8s} {'us/iter':>9s} {'pct':>6s}" + sc_h]
    for g in groups:
        sc = f" {g['us'] * scale:9.2f}" if scale else ""
        out.append(f"{g['level']:6s} {g['phase']:34s} {g['launches']:8.1f} {g['us']:9.2f} {100 * g['us'] / kern:6.2f}"
                   + sc)
    out += ["", f"{'level':6s} {'launches':>8s} {'us/iter':>9s} {'pct':>6s}" + sc_h +
            f" {'nominal_MB':>10s} {'nominal_TB/s':>12s}"]
    by = defaultdict(lambda: [0.0, 0.0])
    for g in groups:
        by[g["level"]][0] += g["launches"]
        by[g["level"]][1] += g["us"]
    for lv in sorted(by, key=lambda v: (v == "CG", v)):
        nl, us = by[lv]
        nb = b["nominal_bytes"].get(lv)
        t = us * scale if scale else us
        rate = f"{nb / (t * 1e-6) / 1e12:12.2f}" if nb else f"{'':12s}"
        mb = f"{nb / 1e6:10.1f}" if nb else f"{'':10s}"
        sc = f" {us * scale:9.2f}" if scale else ""
        out.append(f"{lv:6s} {nl:8.1f} {us:9.2f} {100 * us / kern:6.2f}{sc} {mb} {rate}")
    tot = sum(v[1] for v in by.values())
    out.append(f"{'total':6s} {sum(v[0] for v in by.values()):8.1f} {tot:9.2f} {100.0:6.2f}"
               + (f" {tot * scale:9.2f}" if scale else ""))
    return "\n".join(out)


def iteration_traffic(fetch_dir, write_dir, copy_mib=512):
    """HBM bytes of one CG iteration from the counter runs (see the module doc)."""
    res = {"copy_mib": copy_mib, "kernels": {}}
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    rows.append((int(r.get("Dispatch_Id", r.get("Dispatch_ID", 0))), r["Kernel_Name"],
                                 int(r.get("Grid_Size", r.get("Grid_Size_X", 0))), float(r["Counter_Value"])))
        rows.sort()
        copies = [v for _, n, _, v in rows if "copyBuffer" in n]
        if not copies:
            raise SystemExit(f"{counter}: no copy in {d}")
        factor = copy_mib * 1024.0 / max(copies)
        first = next((k for k, r in enumerate(rows) if _short(r[1]).startswith("k_init_residual")), None)
        if first is None:
            raise SystemExit(f"{counter}: no k_init_residual dispatch in {d}")
        it = [r for r in rows[first + 1:] if _short(r[1]).startswith("k_") and not _short(r[1]).startswith("k_fill")]
        # the initial residual's finalize is set-up, not iteration work
        while it and not _short(it[0][1]).startswith(("k_pass", "k_cast", "k_coarse", "k_restrict")):
            it.pop(0)
        iters = sum(1 for r in it if _short(r[1]).startswith("k_spmv_pq"))
        tot = 0.0
        for _, n, g, v in it:
            b = 1024.0 * v * factor
            tot += b
            k = res["kernels"].setdefault(f"{_short(n)} @{g}", {"calls_per_iteration": 0.0, "fetch": 0.0, "write": 0.0})
            k[tag] += b / iters
            if tag == "fetch":
                k["calls_per_iteration"] += 1.0 / iters
        res[f"{tag}_factor"] = factor
        res[f"{tag}_bytes_per_iteration"] = tot / iters
        res["iterations"] = iters
    res["hbm_bytes_per_iteration"] = res["fetch_bytes_per_iteration"] + res["write_bytes_per_iteration"]
    res["kernel_source_hash"] = kernel_source_hash()
    return res


def iteration_traffic_summary(t, cmd):
    out = ["# HBM bytes of one CG iteration, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs",
           "# (each counter scaled by what it reads for a device copy of known size)",
           f"# commands: {cmd}",
           f"# kernel sources {t['kernel_source_hash']}; {t['iterations']} iterations counted",
           f"# per iteration: read {t['fetch_bytes_per_iteration'] / 1e6:.1f} MB, "
           f"written {t['write_bytes_per_iteration'] / 1e6:.1f} MB, "
           f"total {t['hbm_bytes_per_iteration'] / 1e6:.1f} MB", "",
           f"{'kernel @ grid':70s} {'calls/it':>8s} {'read_MB':>9s} {'write_MB':>9s}"]
    for k, v in sorted(t["kernels"].items(), key=lambda kv: -(kv[1]["fetch"] + kv[1]["write"])):
        out.append(f"{k[:70]:70s} {v['calls_per_iteration']:8.2f} {v['fetch'] / 1e6:9.2f} {v['write'] / 1e6:9.2f}")
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


def counters(dirs, match=None):
    """{(kernel, grid): {counter: [values]}} over one or more --pmc runs"""
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                k = _short(r["Kernel_Name"])
                if match and not re.search(match, k):
                    continue
                g = int(r.get("Grid_Size", r.get("Grid_Size_X", 0)))
                vals[(k, g)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return vals


def counters_summary(vals, cmd, gui_xcds=8, cus=256):
    """Per kernel: dispatches and the mean of every counter per dispatch.  Where
    GRBM_GUI_ACTIVE (summed over the XCDs) was taken, the busy fraction of
    each per-CU unit counter (TA_TA_BUSY, TD_TD_BUSY, summed over the CUs) is
    added: counter / cus / (GRBM_GUI_ACTIVE / xcds)."""
    out = ["# rocprofv3 counter summary: mean per dispatch of every counter, by kernel",
           f"# commands: {cmd}"]
    for (k, g), cs in sorted(vals.items(), key=lambda kv: (-kv[0][1], kv[0][0])):
        n = max(len(v) for v in cs.values())
        mean = {c: sum(v) / len(v) for c, v in cs.items()}
        parts = [f"{c}={m:.4g}" for c, m in sorted(mean.items())]
        gui = mean.get("GRBM_GUI_ACTIVE")
        if gui:
            for c in ("TA_TA_BUSY", "TD_TD_BUSY"):
                if c in mean:
                    parts.append(f"{c}_frac={mean[c] / cus / (gui / gui_xcds):.2f}")
        out.append(f"{k[:64]:64s} grid {g:9d} n {n:4d}  " + " ".join(parts))
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "pmc", "traffic", "traffic-all", "breakdown", "iteration-traffic",
                                     "counters"])
    ap.add_argument("dir")
    ap.add_argument("args", nargs="*")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--json", default=None)
    ap.add_argument("--match", default=None)
    ap.add_argument("--dims", type=int, nargs=3, default=None)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--wall-us", type=float, default=None)
    a = ap.parse_args()
    if a.mode == "breakdown":
        b = breakdown(a.dir, tuple(a.dims), a.levels)
        b["command"] = a.cmd
        b["wall_us_per_iteration"] = a.wall_us
        print(breakdown_summary(b, a.cmd, a.wall_us))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(b, f, indent=1)
                f.write("\n")
        return 0
    if a.mode == "iteration-traffic":
        t = iteration_traffic(a.dir, a.args[0], a.copy_mib)
        t["command"] = a.cmd
        print(iteration_traffic_summary(t, a.cmd))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(t, f, indent=1)
                f.write("\n")
        return 0
    if a.mode == "counters":
        print(counters_summary(counters([a.dir] + a.args, a.match), a.cmd))
        return 0
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
