"""Serving loop: many simulated Lidar sensors, continuous batching on one GPU.

Every sensor registers once: its angle tables and a small pool of frame slots
(device range + label buffers, pinned host label buffers) stay resident,
admitted against an HBM budget.  Frames arrive on their own schedule (Poisson
arrivals at each sensor's rate) in pinned host receive buffers, as a sensor
driver delivers them (here: a pinned pool of frames per sensor).  A frame is admitted as soon as one of its sensor's
slots is free (otherwise it waits, FIFO per sensor); whenever one of the
launch streams is idle, every admitted frame not yet launched (oldest first,
up to max_batch) goes out as one flic_cluster_batched_host call (each frame's
host-to-device copy, the batched launch, each frame's labels back to pinned
host memory) and an event.  Work
from different streams overlaps on the device.  Latency is measured from a
frame's arrival to its labels being on the host.

The loop exists twice.  The library's native serving runtime (flic_server_*,
in C++: serve_native_once, the default) runs admission, FIFO, slots and
continuous batching without the interpreter in the way; ServingCore below is
the same policy in Python, with a backend object doing the copies and
launches.  Its admission, FIFO and statistics logic is tested on the CPU with
a fake backend and a fake clock, and the native runtime is tested against it
event by event (its simulated device completes a launch a fixed time after it
was made).

    python -m paper_2003_00575_amd.serve --seconds 60 --sensors 32 [--loop python]
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import gc
import json
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# Statistics
# ---------------------------------------------------------------------------

def order_stat(xs: Sequence[float], q: float) -> float:
    """Exact order statistic: the smallest x with at least q of the sample <= x."""
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = max(0, math.ceil(q * len(s)) - 1)
    return s[k]


@dataclasses.dataclass
class FrameRecord:
    sensor: int
    frame: int
    t_arrival: float
    t_admit: float = math.nan
    t_launch: float = math.nan
    t_done: float = math.nan
    batch: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


# ---------------------------------------------------------------------------
# Arrivals
# ---------------------------------------------------------------------------

def poisson_schedule(rates_hz: Sequence[float], seconds: float, seed: int,
                     speedup: float = 1.0) -> List[Tuple[float, int, int]]:
    """(time, sensor, frame index) sorted by time; exponential gaps at rate
    rate * speedup per sensor."""
    rng = np.random.default_rng(seed)
    out = []
    for s, f in enumerate(rates_hz):
        t, i = 0.0, 0
        lam = f * speedup
        while True:
            t += rng.exponential(1.0 / lam)
            if t >= seconds:
                break
            out.append((t, s, i))
            i += 1
    out.sort()
    return out


# ---------------------------------------------------------------------------
# Scheduling core
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SensorSpec:
    sensor: int
    H: int
    W: int
    skip_depth: int
    threshold: float

    @property
    def frame_bytes(self) -> int:
        return self.H * self.W * 8          # range in + labels out, on the device


class BudgetError(RuntimeError):
    pass


class ServingCore:
    """Admission, per-sensor FIFO, slot pools and continuous batching.

    backend must provide:
      sensor_bytes(spec) -> int                 resident bytes besides slots
      register(spec, n_slots) -> None           allocate tables + slots
      stage(sensor, slot, frame) -> None        frame data into the slot
      launch(stream, [(sensor, slot)]) -> token enqueue copies + one launch
      done(token) -> bool
      scratch_bytes(max_batch_px) -> int        library scratch for a batch
    and may provide
      ring_bytes(max_batch, spec) -> int        exact device bytes of the
                                                library's launch ring once
                                                reserved for max_batch scans of
                                                the largest shape (preferred)
    """

    def __init__(self, backend, hbm_budget: int, n_streams: int = 3, max_batch: int = 64,
                 slots_per_sensor: int = 3, max_queue: int = 64,
                 clock: Callable[[], float] = time.perf_counter):
        self.b = backend
        self.budget = int(hbm_budget)
        self.n_streams = n_streams
        self.max_batch = max_batch
        self.slots_per_sensor = slots_per_sensor
        self.max_queue = max_queue
        self.clock = clock
        self.specs: Dict[int, SensorSpec] = {}
        self.free_slots: Dict[int, List[int]] = {}
        self.waiting: Dict[int, Deque[FrameRecord]] = {}
        self.admitted: Deque[Tuple[FrameRecord, int]] = collections.deque()
        self.inflight: List[Optional[Tuple[object, List[Tuple[FrameRecord, int]]]]] = [None] * n_streams
        self.records: List[FrameRecord] = []
        self.dropped = 0
        self.batches = 0
        self.reserved = 0

    # -- registration / admission by HBM budget --------------------------------
    def resident_bytes(self, spec: SensorSpec) -> int:
        return self.b.sensor_bytes(spec) + self.slots_per_sensor * spec.frame_bytes

    def scratch_reserve(self) -> int:
        # the library's launch ring: one batch of the largest shapes per stream
        if not self.specs:
            return 0
        biggest = max(self.specs.values(), key=lambda s: s.H * s.W)
        if hasattr(self.b, "ring_bytes"):
            return self.b.ring_bytes(self.max_batch, biggest)
        slots = getattr(self.b, "ring_slots", self.n_streams)
        return self.b.scratch_bytes(self.max_batch * biggest.H * biggest.W) * slots

    def add_sensor(self, spec: SensorSpec) -> None:
        need = self.resident_bytes(spec)
        saved = dict(self.specs)
        self.specs[spec.sensor] = spec
        total = self.reserved + need + self.scratch_reserve()
        if total > self.budget:
            self.specs = saved
            raise BudgetError(f"sensor {spec.sensor}: {total} bytes would exceed the "
                              f"HBM budget of {self.budget}")
        self.b.register(spec, self.slots_per_sensor)
        self.reserved += need
        self.free_slots[spec.sensor] = list(range(self.slots_per_sensor))
        self.waiting[spec.sensor] = collections.deque()

    # -- event handling -------------------------------------------------------------
    def arrive(self, sensor: int, frame: int, t_arrival: float) -> None:
        rec = FrameRecord(sensor, frame, t_arrival)
        self.records.append(rec)
        q = self.waiting[sensor]
        if len(q) >= self.max_queue:
            old = q.popleft()
            old.t_done = math.inf
            self.dropped += 1
        q.append(rec)
        self._admit(sensor)

    def _admit(self, sensor: int) -> None:
        q, slots = self.waiting[sensor], self.free_slots[sensor]
        while q and slots:
            rec = q.popleft()
            slot = slots.pop()
            self.b.stage(sensor, slot, rec.frame)
            rec.t_admit = self.clock()
            self.admitted.append((rec, slot))

    def poll(self) -> int:
        """Retire finished batches; returns how many frames completed."""
        n = 0
        for i, fl in enumerate(self.inflight):
            if fl is None or not self.b.done(fl[0]):
                continue
            now = self.clock()
            for rec, slot in fl[1]:
                rec.t_done = now
                self.free_slots[rec.sensor].append(slot)
                n += 1
            self.inflight[i] = None
            for s in dict.fromkeys(rec.sensor for rec, _ in fl[1]):   # first-appearance order
                self._admit(s)
        return n

    def launch_ready(self) -> int:
        """Launch admitted frames on every idle stream; returns frames launched."""
        n = 0
        for i in range(self.n_streams):
            if self.inflight[i] is not None or not self.admitted:
                continue
            batch = [self.admitted.popleft() for _ in range(min(self.max_batch, len(self.admitted)))]
            now = self.clock()
            for rec, _ in batch:
                rec.t_launch = now
                rec.batch = self.batches
            token = self.b.launch(i, [(rec.sensor, slot) for rec, slot in batch])
            self.inflight[i] = (token, batch)
            self.batches += 1
            n += len(batch)
        return n

    def busy(self) -> bool:
        return bool(self.admitted) or any(f is not None for f in self.inflight) or \
            any(self.waiting[s] for s in self.waiting)

    # -- driver ---------------------------------------------------------------------
    def run(self, schedule: Sequence[Tuple[float, int, int]], drain: bool = True,
            sleep: Callable[[float], None] = time.sleep) -> None:
        """Feed arrivals at their scheduled times (relative to now)."""
        t0 = self.clock()
        i = 0
        while i < len(schedule) or (drain and self.busy()):
            now = self.clock() - t0
            while i < len(schedule) and schedule[i][0] <= now:
                t, s, f = schedule[i]
                self.arrive(s, f, t0 + t)
                i += 1
            self.poll()
            self.launch_ready()
            idle = not self.admitted and all(f is None for f in self.inflight)
            if idle and i < len(schedule):
                wait = schedule[i][0] - (self.clock() - t0)
                if wait > 2e-4:
                    sleep(min(wait, 1e-3))

    def stats(self, warmup_s: float = 0.0, t0: Optional[float] = None) -> dict:
        return frame_stats([(r.sensor, r.t_arrival, r.t_launch, r.t_done) for r in self.records],
                           self.specs, self.dropped, self.batches, warmup_s, t0)


def frame_stats(frames, specs: Dict[int, "SensorSpec"], dropped: int, batches: int,
                warmup_s: float = 0.0, t0: Optional[float] = None) -> dict:
    """Throughput and latency of served frames: frames are (sensor,
    t_arrival, t_launch, t_done) in seconds (t_done infinite when dropped);
    frames that arrived in the first warmup_s seconds after t0 are left out."""
    done = [f for f in frames if math.isfinite(f[3])]
    if t0 is None:
        t0 = min((f[1] for f in frames), default=0.0)
    kept = [f for f in done if f[1] - t0 >= warmup_s]
    lat = [(f[3] - f[1]) * 1e3 for f in kept]
    # launch -> labels on the host: the device part of a frame's latency
    # (copies, kernels, completion seen by the loop), without the queueing
    dev = [(f[3] - f[2]) * 1e3 for f in kept]
    span = (max(f[3] for f in kept) - min(f[1] for f in kept)) if kept else math.nan
    px = sum(specs[f[0]].H * specs[f[0]].W for f in kept)
    return {"frames": len(kept), "dropped": dropped, "batches": batches,
            "p50_ms": order_stat(lat, 0.50), "p99_ms": order_stat(lat, 0.99),
            "launch_p50_ms": order_stat(dev, 0.50), "launch_p99_ms": order_stat(dev, 0.99),
            "max_ms": max(lat) if lat else math.nan,
            "scans_per_s": len(kept) / span if kept and span > 0 else math.nan,
            "gpix_per_s": px / span / 1e9 if kept and span > 0 else math.nan,
            "mean_batch": (len(done) / batches) if batches else 0.0}


# ---------------------------------------------------------------------------
# GPU backend
# ---------------------------------------------------------------------------

def _ring_cap(need: int) -> int:
    """Size of a launch-slot buffer holding `need` bytes: the library grows
    each slot buffer to the next power of two, at least 4 KiB."""
    cap = 4096
    while cap < need:
        cap *= 2
    return cap


class GpuBackend:
    """Device side of the serving loop: resident tables and frame slots,
    copies on the launch streams, batched (or per-scan) launches."""

    ring_slots = 4                         # launch slots of a flic context

    def __init__(self, ctx, frames: Dict[int, List[np.ndarray]], tables: Dict[int, tuple],
                 n_streams: int, batched: bool = True, keep_labels: bool = False):
        import torch
        from . import flic
        self.torch, self.flic = torch, flic
        self.ctx = ctx
        self.frames = frames
        # the sensors' receive buffers: frames arrive in pinned host memory
        self.rx = {s: [torch.from_numpy(np.ascontiguousarray(f)).pin_memory() for f in pool]
                   for s, pool in frames.items()}
        self.tables = tables
        self.batched = batched
        self.keep_labels = keep_labels
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.slots: Dict[Tuple[int, int], dict] = {}
        self.dev_tables: Dict[int, tuple] = {}
        self.specs: Dict[int, SensorSpec] = {}
        self.results: Dict[Tuple[int, int], np.ndarray] = {}

    def sensor_bytes(self, spec: SensorSpec) -> int:
        cv, ch = self.tables[spec.sensor]
        return cv.nbytes + ch.nbytes

    def scratch_bytes(self, px: int) -> int:
        raise NotImplementedError("GpuBackend sizes the launch ring with ring_bytes")

    def _ring_request(self, max_batch: int, spec: SensorSpec) -> Tuple[int, int]:
        """Descriptor and scratch bytes each launch slot is sized for: the
        library's figures for one scan of this shape, times the batch size
        (the block map and scratch grow with every scan of a batch)."""
        flic = self.flic
        # never-dereferenced, non-overlapping addresses: flic_batch_bytes only
        # validates them
        st = flic._Scan(1 << 40, spec.H, spec.W, flic._Tables(3 << 40, 4 << 40), float(spec.threshold),
                        int(spec.skip_depth), 2 << 40)
        desc, scratch = self.ctx.batch_bytes([st])
        n = max(1, max_batch)
        return desc * n, scratch * n

    def ring_bytes(self, max_batch: int, spec: SensorSpec) -> int:
        """Device bytes of the library's launch ring after reserve(): every
        slot's descriptor and scratch buffer, each rounded up to a power of
        two of at least 4 KiB as flic_ctx_reserve sizes them."""
        desc, scratch = self._ring_request(max_batch, spec)
        return self.ring_slots * (_ring_cap(desc) + _ring_cap(scratch))

    def reserve(self, max_batch: int) -> None:
        """Size the library's launch slots for the largest possible batch now,
        so no launch allocates (or frees, which synchronises the device)."""
        biggest = max(self.specs.values(), key=lambda s: s.H * s.W)
        self.ctx.reserve(*self._ring_request(max_batch, biggest))

    def register(self, spec: SensorSpec, n_slots: int) -> None:
        torch = self.torch
        cv, ch = self.tables[spec.sensor]
        dcv = torch.from_numpy(cv).cuda()
        dch = torch.from_numpy(ch).cuda()
        self.dev_tables[spec.sensor] = (dcv, dch)
        self.specs[spec.sensor] = spec
        for k in range(n_slots):
            rng_d = torch.empty((spec.H, spec.W), dtype=torch.float32, device="cuda")
            lab_d = torch.empty((spec.H, spec.W), dtype=torch.int32, device="cuda")
            st = self.flic._Scan(rng_d.data_ptr(), spec.H, spec.W,
                                 self.flic._Tables(dcv.data_ptr(), dch.data_ptr()),
                                 float(spec.threshold), int(spec.skip_depth), lab_d.data_ptr())
            h_out = torch.empty((spec.H, spec.W), dtype=torch.int32, pin_memory=True)
            self.slots[(spec.sensor, k)] = {
                "range": rng_d, "labels": lab_d, "struct": st, "src": 0,
                "h_out": h_out, "out": h_out.data_ptr(), "frame": -1}

    def stage(self, sensor: int, slot: int, frame: int) -> None:
        sl = self.slots[(sensor, slot)]
        rx = self.rx[sensor]
        sl["src"] = rx[frame % len(rx)].data_ptr()   # the receive buffer the frame arrived in
        sl["frame"] = frame

    def launch(self, stream: int, items: Sequence[Tuple[int, int]]):
        import ctypes
        torch = self.torch
        st = self.streams[stream]
        slots = [self.slots[key] for key in items]
        n = len(slots)
        structs = (self.flic._Scan * n)(*[sl["struct"] for sl in slots])
        h_in = (ctypes.c_void_p * n)(*[sl["src"] for sl in slots])
        h_out = (ctypes.c_void_p * n)(*[sl["out"] for sl in slots])
        if self.batched:
            self.ctx.cluster_batched_host(structs, n, h_in, h_out, st)
        else:                                 # one launch sequence (and its copies) per frame
            size = ctypes.sizeof(self.flic._Scan)
            vp = ctypes.sizeof(ctypes.c_void_p)
            for i in range(n):
                self.ctx.cluster_batched_host(
                    ctypes.cast(ctypes.addressof(structs) + i * size, ctypes.POINTER(self.flic._Scan)), 1,
                    ctypes.cast(ctypes.addressof(h_in) + i * vp, ctypes.POINTER(ctypes.c_void_p)),
                    ctypes.cast(ctypes.addressof(h_out) + i * vp, ctypes.POINTER(ctypes.c_void_p)), st)
        ev = torch.cuda.Event()
        ev.record(st)
        return (ev, list(items))

    def done(self, token) -> bool:
        ev, items = token
        if not ev.query():
            return False
        if self.keep_labels:
            for key in items:
                sl = self.slots[key]
                self.results[(key[0], sl["frame"])] = sl["h_out"].numpy().copy()
        return True


# ---------------------------------------------------------------------------
# Workload and runner
# ---------------------------------------------------------------------------

def make_fleet(n_sensors: int, pool: int, seed: int = 0):
    """Sensor s uses the mixed shape s mod 5; rate U(10, 20) Hz; threshold
    U{0.3, 0.5, 0.8, 1.0}; skip depth 3; a pool of raycast frames."""
    from . import synth
    rng = np.random.default_rng(seed)
    specs, frames, tables, rates = [], {}, {}, []
    for s in range(n_sensors):
        H, W, _, _ = synth.MIXED_SHAPES[s % 5]
        T = float(rng.choice([0.3, 0.5, 0.8, 1.0]))
        rates.append(float(rng.uniform(10.0, 20.0)))
        specs.append(SensorSpec(s, H, W, 3, T))
        scans = [synth.sensor_frame(s, f, T) for f in range(pool)]
        frames[s] = [sc.range_img for sc in scans]
        tables[s] = (scans[0].cos_v, scans[0].cos_h)
    return specs, frames, tables, rates


def serve_once(specs, frames, tables, rates, seconds: float, speedup: float, batched: bool,
               n_streams: int, budget: int, seed: int = 1, warmup_s: float = 1.0,
               max_batch: int = 64, keep_labels: bool = False):
    import torch
    from . import flic
    from . import autotune
    ctx = flic.Context(0, hbm_budget_bytes=budget)       # the library enforces the cap on its own buffers
    autotune.apply_default(ctx)
    be = GpuBackend(ctx, frames, tables, n_streams, batched=batched, keep_labels=keep_labels)
    core = ServingCore(be, budget, n_streams=n_streams, max_batch=max_batch if batched else 1)
    for sp in specs:
        core.add_sensor(sp)
    be.reserve(max_batch if batched else 1)
    if ctx.bytes_in_use() > core.scratch_reserve():
        raise BudgetError(f"the library holds {ctx.bytes_in_use()} bytes, admission counted "
                          f"{core.scratch_reserve()}")
    # warm the launch paths before the clock starts
    warm = [(0.0, sp.sensor, 0) for sp in specs]
    core.run(warm)
    torch.cuda.synchronize()
    core.records.clear()
    core.dropped = 0
    core.batches = 0
    sched = poisson_schedule(rates, seconds, seed, speedup)
    gc_was = gc.isenabled()
    gc.disable()                      # no collector pauses inside the timed loop
    try:
        t0 = time.perf_counter()
        core.run(sched)
        torch.cuda.synchronize()
    finally:
        if gc_was:
            gc.enable()
    st = core.stats(warmup_s=warmup_s, t0=t0)
    st.update({"mode": "batched" if batched else "per-scan", "speedup": speedup,
               "streams": n_streams, "offered_scans_per_s": sum(rates) * speedup,
               "hbm_reserved_bytes": core.reserved, "ctx_bytes": ctx.bytes_in_use()})
    return st, be, core


def serve_native_once(specs, frames, tables, rates, seconds: float, speedup: float, batched: bool,
                      n_streams: int, budget: int, seed: int = 1, warmup_s: float = 1.0,
                      max_batch: int = 64, slots_per_sensor: int = 8, max_queue: int = 64,
                      keep_labels: bool = False, schedule=None, copies: str = "kernel"):
    """The same workload served by the library's native runtime
    (flic_server_*): admission, FIFO, slots and continuous batching run in
    C++ inside flic_server_replay, which replays the arrival schedule in real
    time.  With keep_labels every frame gets its own pinned label buffer and
    the labels are returned by (sensor, frame)."""
    import torch
    from . import flic
    from . import autotune
    ctx = flic.Context(0, hbm_budget_bytes=budget)
    autotune.apply_default(ctx)
    srv = flic.Server(ctx, n_streams=n_streams, max_batch=max_batch if batched else 1,
                      slots_per_sensor=slots_per_sensor, max_queue=max_queue, hbm_budget=budget,
                      stage_kernels={"dma": 0, "kernel": 1, "direct": 2}[copies])
    spec_of = {}
    for sp in specs:
        cv, ch = tables[sp.sensor]
        sid = srv.add_sensor(sp.H, sp.W, cv, ch, sp.threshold, sp.skip_depth)
        assert sid == sp.sensor, "sensors are registered in id order"
        spec_of[sp.sensor] = sp
    # receive buffers (frames arrive in pinned host memory) and label buffers
    rx = {s: [torch.from_numpy(np.ascontiguousarray(f)).pin_memory() for f in pool]
          for s, pool in frames.items()}
    ring = slots_per_sensor + 1
    out = {sp.sensor: [torch.empty((sp.H, sp.W), dtype=torch.int32, pin_memory=True) for _ in range(ring)]
           for sp in specs}

    def arrivals(sched, own_buffers):
        a = np.zeros(len(sched), dtype=flic.ARRIVAL_DTYPE)
        kept = {}
        for k, (t, s, f) in enumerate(sched):
            a[k]["t"], a[k]["sensor"] = t, s
            a[k]["host_range"] = rx[s][f % len(rx[s])].data_ptr()
            if own_buffers:
                buf = torch.empty((spec_of[s].H, spec_of[s].W), dtype=torch.int32, pin_memory=True)
                kept[(s, f)] = buf
            else:
                buf = out[s][f % ring]
            a[k]["host_labels"] = buf.data_ptr()
        return a, kept

    warm, _ = arrivals([(0.0, sp.sensor, 0) for sp in specs], False)
    srv.replay(warm)                   # warm the launch paths before the clock starts
    torch.cuda.synchronize()
    srv.clear()
    sched = schedule if schedule is not None else poisson_schedule(rates, seconds, seed, speedup)
    arr, kept = arrivals(sched, keep_labels)
    t0 = srv.now()
    srv.replay(arr)
    torch.cuda.synchronize()
    rec, dropped, launches = srv.records()
    st = frame_stats(list(zip(rec["sensor"].tolist(), rec["t_arrival"].tolist(), rec["t_launch"].tolist(),
                              rec["t_done"].tolist())), spec_of, dropped, launches, warmup_s, t0)
    used = ctx.bytes_in_use()
    st.update({"mode": "batched" if batched else "per-scan", "loop": "native",
               "copies": copies, "speedup": speedup,
               "streams": n_streams, "offered_scans_per_s": sum(rates) * speedup, "ctx_bytes": used})
    labels = {key: buf.numpy().copy() for key, buf in kept.items()} if keep_labels else None
    srv.close()
    return st, labels


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--sensors", type=int, default=32)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--warmup", type=float, default=2.0)
    ap.add_argument("--pool", type=int, default=16, help="frames generated per sensor")
    ap.add_argument("--speedups", default="1,4,16", help="time-compression factors to sweep")
    ap.add_argument("--streams", type=int, default=3)
    ap.add_argument("--budget-gb", type=float, default=4.0)
    ap.add_argument("--p99-ms", type=float, default=10.0)
    ap.add_argument("--loop", choices=("native", "python"), default="native",
                    help="the library's native serving runtime, or this module's Python loop")
    ap.add_argument("--slots", type=int, default=8, help="device frame slots per sensor (native loop)")
    ap.add_argument("--copies", choices=("kernel", "dma", "direct"), default="kernel",
                    help="native loop: one staging kernel per batch and direction, a DMA copy per frame, "
                         "or none (the passes read and write the pinned host buffers)")
    args = ap.parse_args()
    specs, frames, tables, rates = make_fleet(args.sensors, args.pool)
    out = []
    for m in [float(x) for x in args.speedups.split(",")]:
        for batched in (True, False):
            if args.loop == "native":
                st, _ = serve_native_once(specs, frames, tables, rates, args.seconds, m, batched,
                                          args.streams, int(args.budget_gb * 2**30), warmup_s=args.warmup,
                                          copies=args.copies, slots_per_sensor=args.slots)
            else:
                st, _, _ = serve_once(specs, frames, tables, rates, args.seconds, m, batched,
                                      args.streams, int(args.budget_gb * 2**30), warmup_s=args.warmup)
                st["loop"] = "python"
            out.append(st)
            print(json.dumps(st), flush=True)
    for mode in ("batched", "per-scan"):
        ok = [s for s in out if s["mode"] == mode and s["p99_ms"] <= args.p99_ms and s["dropped"] == 0]
        best = max(ok, key=lambda s: s["scans_per_s"]) if ok else None
        print(json.dumps({"mode": mode, "p99_limit_ms": args.p99_ms,
                          "max_scans_per_s_at_p99": best["scans_per_s"] if best else None}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
