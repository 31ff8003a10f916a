"""Summarise rocprofv3 CSV output (kernel statistics and per-dispatch counters).

    python -m paper_2407_04634_amd.rocprof_summary OUTDIR [--kernel REGEX] [--top N] [--split-us T]
                                                   [--grid-x X1,X2,...] [--by-grid]

OUTDIR is a rocprofv3 ``-d`` directory written with ``--output-format csv``.
For ``*_kernel_stats.csv`` it prints calls, average and total duration per
kernel; for ``*_counter_collection.csv`` (``--pmc`` runs) it prints, per kernel
and counter, the number of dispatches and the mean value per dispatch.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
from collections import defaultdict


def _find(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def kernel_stats(path, pat, top):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        name = _find(r, "Name", "KernelName", "Kernel_Name")
        if pat and not re.search(pat, name):
            continue
        out.append((name, int(_find(r, "Calls")), float(_find(r, "AverageNs")),
                    float(_find(r, "TotalDurationNs")), float(_find(r, "Percentage"))))
    out.sort(key=lambda t: -t[3])
    lines = [f"{'calls':>9} {'avg_us':>10} {'total_ms':>10} {'pct':>6}  kernel"]
    for name, calls, avg, tot, pct in out[:top]:
        lines.append(f"{calls:>9d} {avg / 1e3:>10.2f} {tot / 1e6:>10.1f} {pct:>6.2f}  {name[:150]}")
    return "\n".join(lines)


def counters(path, pat, vmin=0.0):
    acc = defaultdict(lambda: [0, 0.0])
    with open(path) as f:
        for r in csv.DictReader(f):
            name = _find(r, "Kernel_Name", "KernelName", "Name")
            if pat and not re.search(pat, name):
                continue
            key = (name, _find(r, "Counter_Name", "CounterName"))
            v = float(_find(r, "Counter_Value", "CounterValue"))
            if v < vmin:
                continue
            a = acc[key]
            a[0] += 1
            a[1] += v
    lines = [f"{'dispatches':>10} {'mean/dispatch':>16}  counter  kernel"
             + (f"  (dispatches with value >= {vmin:g})" if vmin > 0 else "")]
    for (name, cn), (cnt, tot) in sorted(acc.items(), key=lambda kv: (kv[0][1], kv[0][0])):
        lines.append(f"{cnt:>10d} {tot / cnt:>16.1f}  {cn}  {name[:150]}")
    return "\n".join(lines)


def trace_split(path, pat, split_us, grid_x=None):
    """Dispatches of the matching kernels split at ``split_us``: count and mean duration.

    ``grid_x`` (a set of work-item counts) keeps only dispatches whose grid has
    that x extent, e.g. to separate one workload's launches from another's."""
    acc = defaultdict(lambda: [0, 0.0, 0, 0.0])
    with open(path) as f:
        for r in csv.DictReader(f):
            name = _find(r, "Kernel_Name", "KernelName", "Name")
            if pat and not re.search(pat, name):
                continue
            if grid_x and int(float(_find(r, "Grid_Size_X", "Grid_Size", "Grid_X"))) not in grid_x:
                continue
            us = (float(_find(r, "End_Timestamp")) - float(_find(r, "Start_Timestamp"))) / 1e3
            a = acc[name]
            if us >= split_us:
                a[0] += 1
                a[1] += us
            else:
                a[2] += 1
                a[3] += us
    lines = [f"{'long':>9} {'avg_us':>9} {'short':>9} {'avg_us':>9}  kernel (split at {split_us} us"
             + (f", grid x in {sorted(grid_x)})" if grid_x else ")")]
    for name, (nl, tl, ns, ts) in sorted(acc.items()):
        lines.append(f"{nl:>9d} {tl / max(nl, 1):>9.2f} {ns:>9d} {ts / max(ns, 1):>9.2f}  {name[:150]}")
    return "\n".join(lines)


def trace_by_grid(path, pat, top):
    """Dispatches of the matching kernels grouped by grid shape (work-items in
    x and y): count, mean and total duration, the ``top`` shapes by total time."""
    acc = defaultdict(lambda: [0, 0.0])
    with open(path) as f:
        for r in csv.DictReader(f):
            name = _find(r, "Kernel_Name", "KernelName", "Name")
            if pat and not re.search(pat, name):
                continue
            gx = int(float(_find(r, "Grid_Size_X", "Grid_Size", "Grid_X")))
            gy = int(float(_find(r, "Grid_Size_Y", "Grid_Y")))
            us = (float(_find(r, "End_Timestamp")) - float(_find(r, "Start_Timestamp"))) / 1e3
            a = acc[(name, gx, gy)]
            a[0] += 1
            a[1] += us
    lines = [f"{'grid_x':>9} {'grid_y':>7} {'calls':>7} {'avg_us':>9} {'total_ms':>9}  kernel"]
    for (name, gx, gy), (n, t) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"{gx:>9d} {gy:>7d} {n:>7d} {t / n:>9.2f} {t / 1e3:>9.2f}  {name[:120]}")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("outdir")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--top", type=int, default=30)
    ap.add_argument("--counter-min", type=float, default=0.0,
                    help="average counters only over dispatches whose value is at least this")
    ap.add_argument("--split-us", type=float, default=0.0,
                    help="also split the matching kernels' dispatches in *_kernel_trace.csv at this duration")
    ap.add_argument("--grid-x", default="",
                    help="comma-separated grid x extents (work-items) the split keeps")
    ap.add_argument("--by-grid", action="store_true",
                    help="also group the matching kernels' dispatches in *_kernel_trace.csv by grid shape")
    a = ap.parse_args()
    gx = {int(v) for v in a.grid_x.split(",") if v} or None
    for p in sorted(glob.glob(os.path.join(a.outdir, "**", "*kernel_stats.csv"), recursive=True)):
        print(f"== {os.path.basename(p)}")
        print(kernel_stats(p, a.kernel, a.top))
    if a.split_us > 0:
        for p in sorted(glob.glob(os.path.join(a.outdir, "**", "*kernel_trace.csv"), recursive=True)):
            print(f"== {os.path.basename(p)}")
            print(trace_split(p, a.kernel, a.split_us, gx))
    if a.by_grid:
        for p in sorted(glob.glob(os.path.join(a.outdir, "**", "*kernel_trace.csv"), recursive=True)):
            print(f"== {os.path.basename(p)} by grid shape")
            print(trace_by_grid(p, a.kernel, a.top))
    for p in sorted(glob.glob(os.path.join(a.outdir, "**", "*counter_collection.csv"), recursive=True)):
        print(f"== {os.path.basename(p)}")
        print(counters(p, a.kernel))
        if a.counter_min > 0:
            print(counters(p, a.kernel, a.counter_min))


if __name__ == "__main__":
    main()
