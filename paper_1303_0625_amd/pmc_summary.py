"""Summarise rocprofv3 outputs of the lattice time-step kernel.

Two uses:

* ``stats``: from a ``rocprofv3 --kernel-trace --stats -f csv`` run, the
  average duration of the time-step kernel per grid size (one line per
  workload), written as a short text summary;
* ``traffic``: from four ``rocprofv3 --pmc ... -f csv`` runs (FETCH_SIZE and
  WRITE_SIZE of the lattice command, then of ``calibrate_copy``), the HBM bytes
  per launch of the time-step kernel, scaled by what the same counters read for
  a plain copy of known size; written as JSON tagged with the kernel source
  hash (a record taken on other kernel sources is not used by the benchmark).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import statistics

from .build import source_hash


def _rows(d: str, suffix: str):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _get(row: dict, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def counter_per_dispatch(d: str, counter: str, kernel_regex: str, grid=None):
    """Average per dispatch of `counter` over dispatches of matching kernels
    (optionally only those with the given grid size)."""
    per = {}
    rx = re.compile(kernel_regex)
    for r in _rows(d, "counter_collection.csv"):
        if _get(r, "Counter_Name", "Counter") != counter:
            continue
        if not rx.search(_get(r, "Kernel_Name", "Kernel-Name")):
            continue
        if grid is not None and int(float(_get(r, "Grid_Size", "Grid-Size"))) != grid:
            continue
        key = _get(r, "Dispatch_Id", "Dispatch-Id", "Correlation_Id")
        per[key] = per.get(key, 0.0) + float(_get(r, "Counter_Value", "Value"))
    if not per:
        raise ValueError(f"no {counter} samples for /{kernel_regex}/ (grid {grid}) in {d}")
    vals = sorted(per.values())
    return statistics.median(vals), len(vals)


def kernel_durations(d: str, kernel_regex: str):
    """{grid_size: (calls, mean_us, min_us, max_us)} from the kernel trace."""
    rx = re.compile(kernel_regex)
    acc = {}
    for r in _rows(d, "kernel_trace.csv"):
        if not rx.search(_get(r, "Kernel_Name", "Kernel-Name")):
            continue
        g = int(float(_get(r, "Grid_Size", "Grid_Size_X", "Grid-Size")))
        dur = (float(_get(r, "End_Timestamp")) - float(_get(r, "Start_Timestamp"))) / 1000.0
        acc.setdefault(g, []).append(dur)
    return {g: (len(v), statistics.mean(v), min(v), max(v)) for g, v in acc.items()}


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--kernel", default="k_fused")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch-dir", required=True)
    t.add_argument("--write-dir", required=True)
    t.add_argument("--copy-fetch-dir", required=True)
    t.add_argument("--copy-write-dir", required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--kernel", default="k_fused")
    t.add_argument("--copy-kernel", default="copy|elementwise")
    t.add_argument("--grid", type=int, default=None)
    t.add_argument("--workload", required=True)
    t.add_argument("--alg-bytes", type=float, required=True)
    t.add_argument("--commands", required=True)
    t.add_argument("--family", default="lbm", help="kernel source family the hash covers (lbm, lbm3d or nn)")
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        d = kernel_durations(a.dir, a.kernel)
        lines = [f"# {a.kernel} kernel durations (rocprofv3 --kernel-trace --stats)", "",
                 "Command:", "", "```", a.command, "```", "",
                 "| grid size | calls | mean us | min us | max us |", "|---|---|---|---|---|"]
        for g, (n, mean, lo, hi) in sorted(d.items()):
            lines.append(f"| {g} | {n} | {mean:.3f} | {lo:.3f} | {hi:.3f} |")
        os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
        with open(a.out, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        return
    fetch, nf = counter_per_dispatch(a.fetch_dir, "FETCH_SIZE", a.kernel, a.grid)
    write, nw = counter_per_dispatch(a.write_dir, "WRITE_SIZE", a.kernel, a.grid)
    cfetch, _ = counter_per_dispatch(a.copy_fetch_dir, "FETCH_SIZE", a.copy_kernel)
    cwrite, _ = counter_per_dispatch(a.copy_write_dir, "WRITE_SIZE", a.copy_kernel)
    copy_bytes = a.copy_mib * (1 << 20)
    sf = copy_bytes / (cfetch * 1024.0)
    sw = copy_bytes / (cwrite * 1024.0)
    traffic = fetch * 1024.0 * sf + write * 1024.0 * sw
    rec = {
        "kernel": a.kernel, "workload": a.workload, "grid": a.grid,
        "kernel_source_hash": source_hash(a.family), "source_family": a.family,
        "fetch_kib_per_launch": fetch, "write_kib_per_launch": write,
        "copy_fetch_kib": cfetch, "copy_write_kib": cwrite, "copy_bytes_each_way": copy_bytes,
        "scale_fetch": sf, "scale_write": sw,
        "hbm_bytes_per_launch": traffic, "alg_bytes_per_launch": a.alg_bytes,
        "traffic_over_alg": traffic / a.alg_bytes, "dispatches": [nf, nw],
        "commands": a.commands,
    }
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
