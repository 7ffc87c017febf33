"""Summarise rocprofv3 CSV output for this library's kernels.

    python -m paper_2003_00575_amd.prof_summary <rocprofv3 output dir> [...]

Groups dispatches by (kernel, grid size) and prints, per group, the dispatch
count and mean/min duration (from *_kernel_trace.csv) and the mean value per
dispatch of every collected counter (from *_counter_collection.csv).
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import sys


def _short(name: str) -> str:
    name = name.replace("flic::(anonymous namespace)::", "").replace("(flic::BatchRef)", "")
    return name.replace("void ", "")[:60]


def summarize(d: str) -> str:
    out = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        groups = collections.defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                key = (_short(row["Kernel_Name"]), int(row.get("Grid_Size_X", row.get("Grid_Size", 0)) or 0))
                groups[key].append(int(row["End_Timestamp"]) - int(row["Start_Timestamp"]))
        out.append(f"# kernel trace: {os.path.relpath(path, d)}")
        out.append(f"{'kernel':60s} {'grid':>9s} {'n':>5s} {'mean_us':>9s} {'min_us':>9s}")
        for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            out.append(f"{k:60s} {g:9d} {len(v):5d} {sum(v) / len(v) / 1e3:9.2f} {min(v) / 1e3:9.2f}")
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        acc = collections.defaultdict(lambda: collections.defaultdict(float))
        cnt = collections.defaultdict(set)
        with open(path) as f:
            for row in csv.DictReader(f):
                key = (_short(row["Kernel_Name"]), int(row.get("Grid_Size", 0) or 0))
                acc[key][row["Counter_Name"]] += float(row["Counter_Value"])
                cnt[key].add(row.get("Dispatch_Id", row.get("Correlation_Id")))
        out.append(f"# counters (mean per dispatch): {os.path.relpath(path, d)}")
        for key in sorted(acc, key=lambda k: (k[0], k[1])):
            n = max(1, len(cnt[key]))
            vals = "  ".join(f"{c}={v / n:.4g}" for c, v in sorted(acc[key].items()))
            out.append(f"{key[0]:60s} grid={key[1]:<9d} n={n:<4d} {vals}")
    return "\n".join(out)


if __name__ == "__main__":
    for d in sys.argv[1:]:
        print(summarize(d))
