"""Summarise rocprofv3 CSV output into the short text kept under profiles/.

  python -m paper_2507_18282_amd.profsummary trace <kernel_trace.csv> <out.txt> --command "<cmd>"
      per-kernel totals, and per (kernel, grid size) averages so that one level
      of the multigrid hierarchy can be read off directly;
  python -m paper_2507_18282_amd.profsummary pmc <counter_collection.csv> <out.txt> --kernel SUBSTR [...]
      --command "<cmd>"
      mean per dispatch of every counter collected, per (kernel, grid size),
      for the kernels whose names contain one of the substrings;
  python -m paper_2507_18282_amd.profsummary counters <fetch.csv> <write.csv> <out.txt> --kernel SUBSTR
      --grid G --copy-bytes B --command "<cmd>"
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of one kernel at one grid
      size, scaled by what the same counters read for a plain device copy of
      B bytes in the same run (the copy moves B bytes in and B bytes out).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import statistics
import sys


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _grid(r):
    return int(r.get("Grid_Size_X", r.get("Grid_Size", 0)) or 0) * int(r.get("Grid_Size_Y", 1) or 1) * \
        int(r.get("Grid_Size_Z", 1) or 1)


def trace_summary(trace_csv: str, out_txt: str, command: str, top: int = 30) -> None:
    rows = _rows(trace_csv)
    per = collections.defaultdict(list)
    per_grid = collections.defaultdict(list)
    for r in rows:
        name = r["Kernel_Name"]
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per[name].append(d)
        per_grid[(name, _grid(r))].append(d)
    total = sum(sum(v) for v in per.values())
    lines = [f"# rocprofv3 kernel trace summary", f"# command: {command}", f"# dispatches: {len(rows)}",
             f"# total kernel time: {total / 1e6:.3f} ms", "", "## per kernel", "",
             f"{'total_ms':>10} {'share':>6} {'calls':>7} {'avg_us':>9}  kernel"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"{sum(v) / 1e6:10.3f} {100 * sum(v) / total:5.1f}% {len(v):7d} {statistics.mean(v) / 1e3:9.2f}  "
                     f"{name[:120]}")
    lines += ["", "## per kernel and grid size (work-items)", "",
              f"{'total_ms':>10} {'calls':>7} {'avg_us':>9} {'grid':>10}  kernel"]
    for (name, g), v in sorted(per_grid.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"{sum(v) / 1e6:10.3f} {len(v):7d} {statistics.mean(v) / 1e3:9.2f} {g:10d}  {name[:100]}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_per_dispatch(path: str, counter: str):
    """{(kernel name, grid): [values]} for one counter from a rocprofv3 counter_collection.csv."""
    out = collections.defaultdict(list)
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        out[(r["Kernel_Name"], _grid(r))].append(float(r["Counter_Value"]))
    return out


def counter_summary(fetch_csv: str, write_csv: str, out_txt: str, kernel: str, grid: int, copy_bytes: float,
                    command: str, source: str, bytes_alg: float) -> None:
    fetch = _counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _counter_per_dispatch(write_csv, "WRITE_SIZE")

    def pick(d, sub, g):
        vals = [v for (n, gg), vs in d.items() if sub in n and (g is None or gg == g) for v in vs]
        return statistics.mean(vals) if vals else float("nan"), len(vals)

    kf, nf = pick(fetch, kernel, grid)
    kw, nw = pick(write, kernel, grid)
    # the calibration copy is the copy dispatch that moved the most bytes
    cf = max((v for (n, _), vs in fetch.items() if "copyBuffer" in n for v in vs), default=float("nan"))
    cw = max((v for (n, _), vs in write.items() if "copyBuffer" in n for v in vs), default=float("nan"))
    # scale factors: bytes the copy really moved per KiB the counter reported
    sf = copy_bytes / cf if cf == cf and cf > 0 else float("nan")
    sw = copy_bytes / cw if cw == cw and cw > 0 else float("nan")
    fetch_b = kf * sf
    write_b = kw * sw
    with open(source, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    lines = ["# rocprofv3 counter summary (HBM traffic of one kernel)", f"# command: {command}",
             f"# kernel filter: {kernel}, grid {grid}; dispatches: fetch {nf}, write {nw}",
             f"# copy calibration: {copy_bytes:.0f} B copied; FETCH_SIZE {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB",
             f"fetch_kib_per_dispatch = {kf:.1f}", f"write_kib_per_dispatch = {kw:.1f}",
             f"fetch_scale_bytes_per_kib = {sf:.2f}", f"write_scale_bytes_per_kib = {sw:.2f}",
             f"hbm_fetch_bytes_per_launch = {fetch_b:.0f}", f"hbm_write_bytes_per_launch = {write_b:.0f}",
             f"hbm_bytes_per_launch = {fetch_b + write_b:.0f}", f"bytes_alg_per_launch = {bytes_alg:.0f}",
             f"source = {os.path.relpath(source, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))}",
             f"source_sha256_16 = {digest}"]
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def pmc_summary(csv_path: str, out_txt: str, kernels, command: str) -> None:
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    disp = collections.defaultdict(set)
    for r in _rows(csv_path):
        name = r["Kernel_Name"]
        if not any(k in name for k in kernels):
            continue
        key = (name, _grid(r))
        per[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
        disp[key].add(r.get("Dispatch_Id"))
    lines = ["# rocprofv3 counter summary (mean per dispatch)", f"# command: {command}",
             f"# kernel filter: {', '.join(kernels)}", ""]
    for key in sorted(per, key=lambda k: (k[0], k[1])):
        name, grid = key
        lines.append(f"{name[:120]}")
        lines.append(f"  grid {grid}, dispatches {len(disp[key])}")
        for cn in sorted(per[key]):
            vals = per[key][cn]
            lines.append(f"  {cn} = {statistics.mean(vals):.6g}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("trace_csv")
    t.add_argument("out")
    t.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("out")
    c.add_argument("--kernel", required=True)
    c.add_argument("--grid", type=int, default=None)
    c.add_argument("--copy-bytes", type=float, required=True)
    c.add_argument("--bytes-alg", type=float, required=True)
    c.add_argument("--source", required=True)
    c.add_argument("--command", required=True)
    q = sub.add_parser("pmc")
    q.add_argument("csv")
    q.add_argument("out")
    q.add_argument("--kernel", action="append", required=True)
    q.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        trace_summary(a.trace_csv, a.out, a.command)
    elif a.mode == "pmc":
        pmc_summary(a.csv, a.out, a.kernel, a.command)
    else:
        counter_summary(a.fetch_csv, a.write_csv, a.out, a.kernel, a.grid, a.copy_bytes, a.command, a.source,
                        a.bytes_alg)
    return 0


if __name__ == "__main__":
    sys.exit(main())
