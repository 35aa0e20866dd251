"""Summarise rocprofv3 CSV output (kernel statistics and per-kernel counter means).

    python -m paper_2112_14640_amd.rocprof_summary <rocprofv3 output dir> [--match SUBSTRING]

Reads every ``*kernel_stats.csv`` and ``*counter_collection.csv`` under the directory and
prints a short text summary: per kernel the call count and average duration, and per
(kernel, counter) the mean value per dispatch.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os


def summarize(root: str, match: str = "") -> str:
    out = []
    for f in sorted(glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True)):
        rows = [r for r in csv.DictReader(open(f)) if match in r["Name"]]
        rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))
        out.append("# kernel statistics (rocprofv3 --kernel-trace --stats)")
        out.append("calls  avg_us  min_us  max_us  total_ms  kernel")
        for r in rows[:30]:
            out.append(f"{int(r['Calls']):5d} {float(r['AverageNs']) / 1e3:7.1f} {float(r['MinNs']) / 1e3:7.1f} "
                       f"{float(r['MaxNs']) / 1e3:7.1f} {float(r['TotalDurationNs']) / 1e6:9.3f}  {r['Name'][:160]}")
    for f in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True)):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(f)):
            if match in r["Kernel_Name"]:
                agg[(r["Kernel_Name"][:160], r["Counter_Name"])].append(float(r["Counter_Value"]))
        out.append("# counters (mean per dispatch)")
        for (k, c), v in sorted(agg.items()):
            out.append(f"{c:14s} mean={sum(v) / len(v):14.1f} dispatches={len(v):4d}  {k}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("root")
    ap.add_argument("--match", default="")
    a = ap.parse_args()
    print(summarize(a.root, a.match))


if __name__ == "__main__":
    main()
