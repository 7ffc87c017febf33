"""The library's native serving runtime (flic_server_*) on the CPU, with its
simulated device (ctx NULL: a launch is done a fixed time after it was made).

The native scheduler implements the same policy as serve.ServingCore: the two
are driven through the same event sequence with the same clock and must
produce the same history for every frame (admission, launch, batch, done).
Also: budget admission, argument checks, and a real-time replay."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from paper_2003_00575_amd import flic
from paper_2003_00575_amd.serve import SensorSpec, ServingCore, poisson_schedule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class ConstClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FixedLaunchBackend:
    """Each launch is done `dur` seconds (of the shared clock) after it was made."""

    def __init__(self, clock, dur):
        self.clock, self.dur = clock, dur

    def sensor_bytes(self, spec):
        return 0

    def scratch_bytes(self, px):
        return 0

    def register(self, spec, n):
        pass

    def stage(self, sensor, slot, frame):
        pass

    def launch(self, stream, items):
        return self.clock() + self.dur

    def done(self, token):
        return self.clock() >= token


def tables(H, W, N=3):
    return np.full((N, H), 0.9999, np.float32), np.full((N, W), 0.9999, np.float32)


@pytest.mark.parametrize("max_batch,slots,max_queue,streams", [(64, 3, 64, 3), (4, 2, 3, 2), (1, 1, 2, 1)])
def test_native_core_matches_python_core(max_batch, slots, max_queue, streams):
    dur = 2.5e-3
    shapes = [(16, 1024), (32, 1800), (64, 2048), (16, 1024)]
    rates = [400.0, 900.0, 1500.0, 700.0]          # heavy enough to queue, batch and drop
    sched = poisson_schedule(rates, 0.12, seed=11)
    clk = ConstClock()
    core = ServingCore(FixedLaunchBackend(clk, dur), 1 << 40, n_streams=streams, max_batch=max_batch,
                       slots_per_sensor=slots, max_queue=max_queue, clock=clk)
    srv = flic.Server(None, n_streams=streams, max_batch=max_batch, slots_per_sensor=slots,
                      max_queue=max_queue, sim_launch_s=dur)
    for s, (H, W) in enumerate(shapes):
        core.add_sensor(SensorSpec(s, H, W, 3, 0.5))
        assert srv.add_sensor(H, W, *tables(H, W), 0.5, 3) == s
    # events: every arrival, plus a progress tick every 0.3 ms
    ticks = [k * 3e-4 for k in range(int(0.2 / 3e-4))]
    events = sorted([(t, 0, s, f) for t, s, f in sched] + [(t, 1, -1, -1) for t in ticks])
    for t, kind, s, f in events:
        clk.t = t
        if kind == 0:
            core.arrive(s, f, t)
            srv.submit(t, t, s, tag=f)
        else:
            core.poll()
            core.launch_ready()
            srv.progress(t)
    rec, dropped, launches = srv.records()
    assert len(rec) == len(core.records) == len(sched)
    assert dropped == core.dropped and launches == core.batches
    assert launches > 0
    if max_queue <= 3:
        assert dropped > 0                              # the short queues overflow
    for r, py in zip(rec, core.records):
        assert (int(r["sensor"]), int(r["tag"])) == (py.sensor, py.frame)
        assert int(r["batch"]) == py.batch
        for k in ("t_arrival", "t_admit", "t_launch", "t_done"):
            a, b = float(r[k]), getattr(py, k)
            assert (math.isnan(a) and math.isnan(b)) or a == b, (k, a, b)
    done = rec[np.isfinite(rec["t_done"])]
    assert len(done) > 0
    assert np.all(done["t_arrival"] <= done["t_admit"])
    assert np.all(done["t_admit"] <= done["t_launch"])
    assert np.all(done["t_done"] - done["t_launch"] >= dur)
    # no more frames of a sensor in flight than it has slots
    for s in range(len(shapes)):
        ds = done[done["sensor"] == s]
        for t in np.unique(ds["t_launch"]):
            inflight = np.sum((ds["t_launch"] <= t) & (ds["t_done"] > t))
            assert inflight <= slots
    if max_batch == 1:
        assert np.all(np.bincount(done["batch"]) <= 1)


def test_budget_admission():
    H, W, N, slots = 32, 1800, 3, 2
    per_sensor = N * (H + W) * 4 + slots * H * W * 8
    srv = flic.Server(None, slots_per_sensor=slots, hbm_budget=2 * per_sensor, sim_launch_s=1e-3)
    assert srv.add_sensor(H, W, *tables(H, W), 0.5, N) == 0
    assert srv.add_sensor(H, W, *tables(H, W), 0.5, N) == 1
    with pytest.raises(flic.FlicError) as e:
        srv.add_sensor(16, 1024, *tables(16, 1024), 0.5, N)
    assert e.value.status == flic.FLIC_ENOMEM
    srv.submit(0.0, 0.0, 1)
    with pytest.raises(flic.FlicError):
        srv.submit(0.0, 0.0, 2)                        # the refused sensor does not exist


@pytest.mark.parametrize("kw", [dict(n_streams=0), dict(n_streams=9), dict(max_batch=0), dict(max_batch=1025),
                                dict(slots_per_sensor=0), dict(slots_per_sensor=17), dict(max_queue=0),
                                dict(sim_launch_s=-1.0), dict(sim_launch_s=float("inf")),
                                dict(stage_kernels=3), dict(stage_kernels=-1)])
def test_config_checked(kw):
    with pytest.raises(flic.FlicError) as e:
        flic.Server(None, **kw)
    assert e.value.status == flic.FLIC_EINVAL


def test_argument_checks():
    srv = flic.Server(None, sim_launch_s=1e-3)
    for H, W, N, T in [(0, 64, 3, 0.5), (16, 6, 3, 0.5), (16, 64, 0, 0.5), (16, 64, 9, 0.5),
                       (16, 64, 3, -1.0), (16, 64, 3, float("nan"))]:
        with pytest.raises(flic.FlicError):
            srv.add_sensor(H, W, *tables(max(H, 1), W, max(1, min(N, 8))), T, N)
    s = srv.add_sensor(16, 64, *tables(16, 64), 0.5, 3)
    with pytest.raises(flic.FlicError):
        srv.submit(0.0, 0.0, s + 1)
    srv.submit(0.0, 0.0, s)
    with pytest.raises(flic.FlicError):
        srv.clear()                                     # a frame is admitted
    srv.progress(0.0)
    srv.progress(0.01)
    srv.clear()
    rec, dropped, launches = srv.records()
    assert len(rec) == 0 and dropped == 0 and launches == 0
    bad = np.zeros(2, dtype=flic.ARRIVAL_DTYPE)
    bad["t"] = [0.2, 0.1]
    with pytest.raises(flic.FlicError):
        srv.replay(bad)                                 # times must not decrease
    L = flic.lib()
    assert L.flic_server_create(None, None, None) == flic.FLIC_EINVAL
    assert L.flic_server_progress(None, 0.0, None) == flic.FLIC_EINVAL


def test_replay_in_real_time():
    dur = 2e-3
    srv = flic.Server(None, n_streams=2, max_batch=8, sim_launch_s=dur)
    for H, W in [(16, 1024), (32, 1800)]:
        srv.add_sensor(H, W, *tables(H, W), 0.5, 3)
    a = np.zeros(40, dtype=flic.ARRIVAL_DTYPE)
    a["t"] = np.linspace(0.0, 0.06, 40)
    a["sensor"] = np.arange(40) % 2
    t0 = srv.now()
    srv.replay(a)
    rec, dropped, launches = srv.records()
    assert dropped == 0 and len(rec) == 40 and launches >= 1
    assert np.all(np.isfinite(rec["t_done"]))
    assert np.all(rec["t_arrival"] >= t0)
    np.testing.assert_allclose(np.diff(rec["t_arrival"]), np.diff(a["t"]), atol=1e-9)
    assert np.all(rec["t_done"] - rec["t_launch"] >= dur)
    assert np.all(rec["t_admit"] >= rec["t_arrival"]) and np.all(rec["t_launch"] >= rec["t_admit"])
    assert list(rec["tag"]) == list(range(40))


@pytest.mark.parametrize("name,fields", [("flic_server_config", flic._ServerConfig),
                                         ("flic_frame_record", flic._FrameRecord),
                                         ("flic_arrival", flic._Arrival)])
def test_server_struct_layouts_match_header(tmp_path, name, fields):
    names = [f for f, _ in fields._fields_]
    body = "\n".join(f'    printf("%zu\\n", offsetof({name}, {f}));' for f in names)
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "flic.h"\nint main(void) {\n'
                   f'    printf("%zu\\n", sizeof({name}));\n{body}\n    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(fields)] + [getattr(fields, f).offset for f in names]
    assert got == want
    dt = np.dtype(flic.RECORD_DTYPE if name == "flic_frame_record" else
                  flic.ARRIVAL_DTYPE if name == "flic_arrival" else [("x", "u1")])
    if name != "flic_server_config":
        assert dt.itemsize == ctypes.sizeof(fields)
        assert [dt.fields[f][1] for f in names] == want[1:]
