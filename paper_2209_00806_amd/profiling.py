"""Summaries of rocprofv3 output for the TBPM kernels.

* ``stats``: a rocprofv3 ``--kernel-trace --stats --output-format csv``
  ``*_kernel_stats.csv`` -> a short markdown table (calls, average and total
  duration per kernel).
* ``traffic``: two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs (per
  dispatch, KiB) -> HBM bytes per launch of one kernel, each counter scaled by
  what it reads for the library's streaming copy of a known size.  The result
  is stored with a hash of the kernel source, so a consumer can tell whether
  the kernel has changed since the counters were taken.

    python -m paper_2209_00806_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
    python -m paper_2209_00806_amd.profiling trace <kernel_trace.csv | results.db> <out.md> "<command>"
    python -m paper_2209_00806_amd.profiling traffic <fetch.csv> <write.csv> <copy_bytes> \
        <kernel_regex> <kernel_sources,comma,separated> <out.json> "<command>" [grid]
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _col(row, *names):
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return row[k]
    raise KeyError(names)


def stats(csv_path: str, out_md: str, command: str, top: int = 20) -> str:
    rows = _rows(csv_path)
    recs = []
    for r in rows:
        name = _col(r, "Name", "KernelName", "Kernel_Name")
        calls = int(float(_col(r, "Calls")))
        total = float(_col(r, "TotalDurationNs", "Total_Duration_ns", "TotalDuration"))
        avg = float(_col(r, "AverageNs", "Average_ns", "Average"))
        pct = float(_col(r, "Percentage", "Percent"))
        recs.append((total, name, calls, avg, pct))
    recs.sort(reverse=True)
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | average (us) | total (ms) | % |", "|---|---|---|---|---|"]
    for total, name, calls, avg, pct in recs[:top]:
        short = name.replace("tbpm::(anonymous namespace)::", "").replace("(tbpm::PassParams)", "")
        lines.append(f"| `{short}` | {calls} | {avg / 1e3:.2f} | {total / 1e6:.2f} | {pct:.2f} |")
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as fh:
        fh.write(text)
    return text


def _dispatches(path: str):
    """(kernel name, grid threads, duration ns) of every dispatch in a
    ``*_kernel_trace.csv`` or in a rocprofv3 ``*_results.db`` (its default
    output format)."""
    if path.endswith(".db"):
        import sqlite3
        db = sqlite3.connect(path)
        try:
            q = "select name, grid_x * grid_y * grid_z, end - start from kernels"
            return [(n, int(g), int(d)) for n, g, d in db.execute(q)]
        finally:
            db.close()
    out = []
    for r in _rows(path):
        grid = int(_col(r, "Grid_Size_X")) * int(_col(r, "Grid_Size_Y")) * int(_col(r, "Grid_Size_Z"))
        out.append((_col(r, "Kernel_Name"), grid,
                    int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))))
    return out


def trace(csv_path: str, out_md: str, command: str, top: int = 24) -> str:
    """Per (kernel, grid size) statistics from a ``*_kernel_trace.csv`` or a
    ``*_results.db``."""
    groups = {}
    for name, grid, dur in _dispatches(csv_path):
        groups.setdefault((name, grid), []).append(dur)
    total_all = sum(sum(v) for v in groups.values())
    recs = sorted(((sum(v), k, v) for k, v in groups.items()), reverse=True)
    lines = ["# rocprofv3 kernel trace, grouped by kernel and grid size", "", "Command:", "", "```", command, "```",
             "", "| kernel | grid (threads) | calls | average (us) | min (us) | max (us) | total (ms) | % |",
             "|---|---|---|---|---|---|---|---|"]
    for tot, (name, grid), v in recs[:top]:
        short = name.replace("tbpm::(anonymous namespace)::", "").replace("(tbpm::PassParams)", "")
        short = re.sub(r"\(.*\)$", "", short) if not short.startswith("void tbpm") else short
        lines.append(f"| `{short[:110]}` | {grid} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {min(v) / 1e3:.2f} | "
                     f"{max(v) / 1e3:.2f} | {tot / 1e6:.2f} | {100.0 * tot / total_all:.2f} |")
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as fh:
        fh.write(text)
    return text


def _per_dispatch(path: str, counter: str, regex: str, grid: int | None = None):
    vals = {}
    for r in _rows(path):
        if _col(r, "Counter_Name", "CounterName") != counter:
            continue
        name = _col(r, "Kernel_Name", "KernelName")
        if not re.search(regex, name):
            continue
        if grid is not None and int(_col(r, "Grid_Size")) != grid:
            continue
        did = _col(r, "Dispatch_Id", "DispatchId")
        vals[did] = vals.get(did, 0.0) + float(_col(r, "Counter_Value", "CounterValue"))
    return list(vals.values())


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(fetch_csv: str, write_csv: str, copy_bytes: int, kernel_regex: str, kernel_sources,
            out_json: str, command: str, copy_regex: str = r"k_copy", grid: int | None = None) -> dict:
    cf = _per_dispatch(fetch_csv, "FETCH_SIZE", copy_regex)
    cw = _per_dispatch(write_csv, "WRITE_SIZE", copy_regex)
    kf = _per_dispatch(fetch_csv, "FETCH_SIZE", kernel_regex, grid)
    kw = _per_dispatch(write_csv, "WRITE_SIZE", kernel_regex, grid)
    if not (cf and cw and kf and kw):
        raise RuntimeError("missing dispatches in the counter files")
    mean = lambda xs: sum(xs) / len(xs)
    # counters are in KiB per dispatch; scale each by the copy of known size
    fetch_scale = copy_bytes / (mean(cf) * 1024.0)
    write_scale = copy_bytes / (mean(cw) * 1024.0)
    fetch_b = mean(kf) * 1024.0 * fetch_scale
    write_b = mean(kw) * 1024.0 * write_scale
    rec = {"kernel_regex": kernel_regex, "kernel_hash": source_hash(kernel_sources),
           "bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b, "write_bytes": write_b,
           "fetch_scale": fetch_scale, "write_scale": write_scale, "dispatches": [len(kf), len(kw)],
           "copy_bytes_each_way": copy_bytes, "grid": grid, "command": command}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "trace":
        print(trace(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "traffic":
        srcs = sys.argv[6].split(",")
        grid = int(sys.argv[9]) if len(sys.argv) > 9 else None
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], srcs, sys.argv[7],
                                 sys.argv[8], grid=grid), indent=1))
    else:
        raise SystemExit(__doc__)
