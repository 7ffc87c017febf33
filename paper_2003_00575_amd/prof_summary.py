"""Summarise rocprofv3 CSV output for this library's kernels.

    python -m paper_2003_00575_amd.prof_summary <rocprofv3 output dir> [...]

Groups dispatches by (kernel, grid size) and prints, per group, the dispatch
count and mean/min duration (from *_kernel_trace.csv) and the mean value per
dispatch of every collected counter (from *_counter_collection.csv).

    python -m paper_2003_00575_amd.prof_summary --record OUT.txt --workload TEXT \\
        --kernel-trace DIR --fetch DIR --write DIR [--sq DIR] --command CMD [...]

writes one record for a workload: mean kernel durations, HBM bytes per
dispatch from FETCH_SIZE and WRITE_SIZE (each scaled by what the counter reads
for the 128 MiB device copy the profiled program runs once), optional counter
passes (--sq, repeatable: SQ instructions, TCC hits and atomics, occupancy),
the commands that produced the inputs, the SHA-256 of the kernel source, and a
final "json:" line that bench.py reads.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "flic_kernels.hip")
GROUND_SOURCE = os.path.join(HERE, "csrc", "flic_ground.hip")
COPY_BYTES = 128 << 20          # the calibration copy: 128 MiB read, 128 MiB written
PASSES = (("tile_label", "k_tile_label"), ("border_merge", "k_border_unite"), ("border_final", "k_border_final"),
          ("relabel", "k_relabel"),
          ("ground", "k_ground"))


def _short(name: str) -> str:
    name = name.replace("flic::(anonymous namespace)::", "").replace("(flic::BatchRef)", "")
    return name.replace("void ", "")[:60]


def kernel_source_sha256(path: str = KERNEL_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def source_sha_for(pass_name: str) -> str:
    """SHA-256 of the source file that holds the named pass's kernel."""
    return kernel_source_sha256(GROUND_SOURCE if pass_name == "ground" else KERNEL_SOURCE)


def durations(d: str) -> dict:
    """(kernel, grid) -> list of durations in ns."""
    groups = collections.defaultdict(list)
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        with open(path) as f:
            for row in csv.DictReader(f):
                key = (_short(row["Kernel_Name"]), int(row.get("Grid_Size_X", row.get("Grid_Size", 0)) or 0))
                groups[key].append(int(row["End_Timestamp"]) - int(row["Start_Timestamp"]))
    return groups


def counters(d: str) -> dict:
    """(kernel, grid) -> {counter: mean value per dispatch}."""
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    cnt = collections.defaultdict(set)
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(path) as f:
            for row in csv.DictReader(f):
                key = (_short(row["Kernel_Name"]), int(row.get("Grid_Size", 0) or 0))
                acc[key][row["Counter_Name"]] += float(row["Counter_Value"])
                cnt[key].add(row.get("Dispatch_Id", row.get("Correlation_Id")))
    return {k: {c: v / max(1, len(cnt[k])) for c, v in acc[k].items()} for k in acc}


def summarize(d: str) -> str:
    out = []
    groups = durations(d)
    if groups:
        out.append(f"# kernel trace: {d}")
        out.append(f"{'kernel':60s} {'grid':>9s} {'n':>5s} {'mean_us':>9s} {'min_us':>9s}")
        for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
            out.append(f"{k:60s} {g:9d} {len(v):5d} {sum(v) / len(v) / 1e3:9.2f} {min(v) / 1e3:9.2f}")
    cs = counters(d)
    if cs:
        out.append(f"# counters (mean per dispatch): {d}")
        for key in sorted(cs):
            vals = "  ".join(f"{c}={v:.4g}" for c, v in sorted(cs[key].items()))
            out.append(f"{key[0]:60s} grid={key[1]:<9d} {vals}")
    return "\n".join(out)


def _calibration_copy(cs: dict, counter: str):
    """The 128 MiB copy: the copyBuffer dispatch group with the largest reading."""
    best = None
    for (k, g), vals in cs.items():
        if "copyBuffer" in k and counter in vals and (best is None or vals[counter] > best[1]):
            best = ((k, g), vals[counter])
    if best is None:
        raise SystemExit(f"no calibration copy with {counter} found")
    return best


def _pass_key(keys, prefix):
    hits = [k for k in keys if k[0].startswith(prefix)]
    if not hits:
        return None
    return max(hits, key=lambda k: k[1])            # the large-batch launch has the largest grid


def record(args) -> str:
    kt = durations(args.kernel_trace)
    fe = counters(args.fetch)
    wr = counters(args.write)
    # instruction / cache / occupancy counters: one or more passes, merged
    sq_dirs = [args.sq] if isinstance(args.sq, str) else list(args.sq or [])
    sq = {}
    for d in sq_dirs:
        for key, vals in counters(d).items():
            sq.setdefault(key, {}).update(vals)
    (_, fetch_copy_kib) = _calibration_copy(fe, "FETCH_SIZE")
    (_, write_copy_kib) = _calibration_copy(wr, "WRITE_SIZE")
    f_fetch = COPY_BYTES / (fetch_copy_kib * 1024.0)
    f_write = COPY_BYTES / (write_copy_kib * 1024.0)
    kernels = {}
    for short, prefix in PASSES:
        key = _pass_key(kt.keys(), prefix)
        if key is None:
            continue
        v = kt[key]
        fkey = _pass_key(fe.keys(), prefix)
        wkey = _pass_key(wr.keys(), prefix)
        fb = fe[fkey]["FETCH_SIZE"] * 1024.0 * f_fetch if fkey else None
        wb = wr[wkey]["WRITE_SIZE"] * 1024.0 * f_write if wkey else None
        entry = {"kernel": key[0], "grid": key[1], "dispatches": len(v),
                 "mean_us": round(sum(v) / len(v) / 1e3, 3), "min_us": round(min(v) / 1e3, 3),
                 "fetch_bytes": None if fb is None else int(fb),
                 "write_bytes": None if wb is None else int(wb),
                 "traffic_bytes": None if fb is None or wb is None else int(fb + wb)}
        skey = _pass_key(sq.keys(), prefix)
        if skey:
            entry["sq"] = {c: round(x, 1) for c, x in sorted(sq[skey].items())}
        kernels[short] = entry
    sha = kernel_source_sha256()
    gsha = kernel_source_sha256(GROUND_SOURCE)
    lines = [f"# rocprofv3 record: {args.workload}",
             "# commands (repository root; the profiled program is bench.py):"]
    lines += [f"#   {c}" for c in args.command]
    lines += [f"# kernel source: paper_2003_00575_amd/csrc/flic_kernels.hip sha256 {sha}",
              f"# ground kernel source: paper_2003_00575_amd/csrc/flic_ground.hip sha256 {gsha}",
              f"# byte calibration (plain 128 MiB device copy in the same program): FETCH_SIZE "
              f"{fetch_copy_kib:.0f} KiB -> x{f_fetch:.3f}, WRITE_SIZE {write_copy_kib:.0f} KiB -> x{f_write:.3f}",
              "",
              f"{'pass':13s} {'kernel':24s} {'grid':>9s} {'n':>4s} {'mean_us':>8s} {'min_us':>8s} "
              f"{'fetch_MiB':>9s} {'write_MiB':>9s}"]
    for short, e in kernels.items():
        fm = "-" if e["fetch_bytes"] is None else f"{e['fetch_bytes'] / 2**20:.1f}"
        wm = "-" if e["write_bytes"] is None else f"{e['write_bytes'] / 2**20:.1f}"
        lines.append(f"{short:13s} {e['kernel']:24s} {e['grid']:9d} {e['dispatches']:4d} {e['mean_us']:8.2f} "
                     f"{e['min_us']:8.2f} {fm:>9s} {wm:>9s}")
    if sq:
        lines += ["", "counters per dispatch (SQ instructions and waits, TCC hits / misses / atomics, occupancy):"]
        for short, e in kernels.items():
            if "sq" in e:
                lines.append(f"{short:13s} " + "  ".join(f"{c}={x:.4g}" for c, x in e["sq"].items()))
    lines += ["", "json: " + json.dumps({"workload": args.workload, "kernel_source_sha256": sha,
                                          "ground_source_sha256": gsha,
                                          "fetch_factor": round(f_fetch, 4), "write_factor": round(f_write, 4),
                                          "kernels": kernels}, sort_keys=True)]
    return "\n".join(lines) + "\n"


def load_record(path: str):
    """The json line of a record, or None if the file is absent."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("json: "):
                return json.loads(line[len("json: "):])
    return None


def main(argv=None) -> int:
    argv = sys.argv[1:] if argv is None else argv
    if not argv or argv[0] != "--record":
        for d in argv:
            print(summarize(d))
        return 0
    ap = argparse.ArgumentParser()
    ap.add_argument("--record", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--kernel-trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--sq", action="append", default=[],
                    help="a directory of counter passes (repeatable; all are merged per kernel)")
    ap.add_argument("--command", action="append", default=[])
    args = ap.parse_args(argv)
    text = record(args)
    with open(args.record, "w") as f:
        f.write(text)
    print(text)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
