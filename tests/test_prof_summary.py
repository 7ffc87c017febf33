"""The rocprofv3 record builder behind bench.py's roofline.traffic: copy
calibration of FETCH_SIZE / WRITE_SIZE, the largest-grid dispatch chosen per
pass, byte arithmetic, and the source-hash gate bench.py applies."""
import argparse
import csv
import json
import os
import sys

import pytest

from paper_2003_00575_amd import prof_summary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

TILE = "void flic::(anonymous namespace)::k_tile_label<64, 3, false, false>(flic::BatchRef)"
GROUND = "void flic::(anonymous namespace)::k_ground<4>(flic::GroundArgs)"
COPY = "__amd_rocclr_copyBuffer"


def _trace(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "1_kernel_trace.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"])
        for name, grid, us in rows:
            w.writerow([name, grid, 1000, 1000 + int(us * 1000)])


def _counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "1_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for i, (name, grid, kib) in enumerate(rows):
            w.writerow([i, name, grid, counter, kib])


@pytest.fixture
def record(tmp_path):
    kt, fe, wr = str(tmp_path / "kt"), str(tmp_path / "fe"), str(tmp_path / "wr")
    _trace(kt, [(TILE, 2097152, 64.0), (TILE, 2097152, 66.0), (TILE, 16384, 5.0), (GROUND, 16384, 35.0),
                (COPY, 1024, 3.0)])
    # the 128 MiB copy reads as 64 MiB of FETCH_SIZE and 128 MiB of WRITE_SIZE
    _counters(fe, "FETCH_SIZE", [(COPY, 131072, 65536.0), (COPY, 64, 4.0), (TILE, 2097152, 34000.0),
                                 (TILE, 16384, 10.0), (GROUND, 16384, 32000.0)])
    _counters(wr, "WRITE_SIZE", [(COPY, 131072, 131072.0), (TILE, 2097152, 24000.0), (GROUND, 16384, 80000.0)])
    out = str(tmp_path / "rec.txt")
    args = argparse.Namespace(record=out, workload="test", kernel_trace=kt, fetch=fe, write=wr, sq=None,
                              command=["cmd"])
    with open(out, "w") as f:
        f.write(prof_summary.record(args))
    return out


def test_record_bytes_and_pass_choice(record):
    rec = prof_summary.load_record(record)
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    tile = rec["kernels"]["tile_label"]
    assert tile["grid"] == 2097152 and tile["dispatches"] == 2
    assert tile["mean_us"] == pytest.approx(65.0)
    assert tile["fetch_bytes"] == 34000 * 1024 * 2 and tile["write_bytes"] == 24000 * 1024
    assert tile["traffic_bytes"] == tile["fetch_bytes"] + tile["write_bytes"]
    g = rec["kernels"]["ground"]
    assert g["fetch_bytes"] == 32000 * 1024 * 2 and g["write_bytes"] == 80000 * 1024
    assert rec["kernel_source_sha256"] == prof_summary.kernel_source_sha256()
    assert rec["ground_source_sha256"] == prof_summary.kernel_source_sha256(prof_summary.GROUND_SOURCE)


def test_bench_gates_on_source_hash(record, tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    assert bench.dominant_traffic("tile_label", record)["traffic_bytes"] > 0
    assert bench.dominant_traffic("ground", record)["traffic_bytes"] > 0
    text = open(record).read()
    rec = prof_summary.load_record(record)
    stale = str(tmp_path / "stale.txt")
    with open(stale, "w") as f:
        f.write(text.replace(rec["kernel_source_sha256"], "0" * 64))
    assert bench.dominant_traffic("tile_label", stale) is None
    assert bench.dominant_traffic("ground", stale)["traffic_bytes"] > 0      # its own source unchanged
    assert bench.dominant_traffic("tile_label", str(tmp_path / "missing.txt")) is None

