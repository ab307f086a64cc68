"""Small summaries of rocprofv3 output for the library's kernels: kernel-trace
durations and hardware-counter values per dispatch, reduced to a few numbers
that can be kept beside the code (the raw CSV of a sweep run holds thousands
of dispatches).

    python -m paper_1612_00595_amd.profiling trace DIR --kernel k_sweep_color --last 180
    python -m paper_1612_00595_amd.profiling counters DIR --kernel k_sweep_color --last 180

DIR is a rocprofv3 output directory written with --output-format csv.  The
last N dispatches of the kernels whose name contains the pattern are
summarised (the timed sweeps come last in the measurement runs); `counters`
also reports the first device copy kernel's values, the calibration of byte
counters against a copy of known size.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import sys


def _files(d: str, suffix: str) -> list[str]:
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def trace(d: str, pattern: str, last: int, top: int = 12) -> dict:
    rows = []
    for f in _files(d, "kernel_trace.csv"):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    by = collections.defaultdict(list)
    for a, b, n in rows:
        by[n].append(b - a)
    top = sorted(by.items(), key=lambda kv: -sum(kv[1]))[:top]
    sel = [b - a for a, b, n in rows if pattern in n][-last:]
    return {
        "pattern": pattern,
        "dispatches": len(sel),
        "mean_us": sum(sel) / len(sel) / 1e3 if sel else None,
        "min_us": min(sel) / 1e3 if sel else None,
        "max_us": max(sel) / 1e3 if sel else None,
        "by_kernel": [{"kernel": n[:120], "calls": len(v), "mean_us": sum(v) / len(v) / 1e3,
                       "total_ms": sum(v) / 1e6} for n, v in top],
    }


def counters(d: str, pattern: str, last: int) -> dict:
    per = collections.OrderedDict()   # dispatch id -> (name, {counter: value})
    for f in _files(d, "counter_collection.csv"):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                key = (f, int(r["Dispatch_Id"]))
                name, vals = per.setdefault(key, (r["Kernel_Name"], {}))
                vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    items = list(per.values())
    sel = [v for n, v in items if pattern in n][-last:]
    names = sorted({c for v in sel for c in v})
    out = {"pattern": pattern, "dispatches": len(sel),
           "mean_per_dispatch": {c: sum(v.get(c, 0.0) for v in sel) / max(len(sel), 1)
                                 for c in names}}
    copies = [v for n, v in items if "copyBuffer" in n or "copy" in n.lower()]
    if copies:
        big = max(copies, key=lambda v: max(v.values()) if v else 0.0)
        out["largest_copy_dispatch"] = big
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters"])
    ap.add_argument("dir")
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--last", type=int, default=1 << 30)
    ap.add_argument("--top", type=int, default=12, help="kernels listed by total time")
    a = ap.parse_args(argv)
    res = trace(a.dir, a.kernel, a.last, a.top) if a.mode == "trace" else counters(a.dir, a.kernel,
                                                                            a.last)
    json.dump(res, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
