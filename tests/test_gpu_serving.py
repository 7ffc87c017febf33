"""Serving loop and autotuner on the GPU.

Alone vs in the mix: every frame served by the continuous-batching loop (many
sensors, mixed shapes, overlapping streams) must carry exactly the labels the
oracle gives for that frame alone, and the labels the plain per-scan path
gives.  The autotuner's tile rules change speed only, never labels."""
import numpy as np
import pytest

import oracle
from paper_2003_00575_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def flic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_00575_amd import flic as f
    f.lib()
    return f


@pytest.mark.parametrize("batched", [True, False])
def test_served_frames_equal_alone(flic, batched):
    from paper_2003_00575_amd import serve
    specs, frames, tables, rates = serve.make_fleet(10, pool=3, seed=5)
    st, be, core = serve.serve_once(specs, frames, tables, rates, seconds=0.4, speedup=4.0,
                                    batched=batched, n_streams=3, budget=4 << 30,
                                    warmup_s=0.0, keep_labels=True)
    assert st["frames"] > 20 and st["dropped"] == 0
    if batched:
        assert st["mean_batch"] > 1.0
    checked = 0
    for (sensor, frame), got in sorted(be.results.items()):
        sp = specs[sensor]
        pool = frames[sensor]
        img = pool[frame % len(pool)]
        cv, ch = tables[sensor]
        want = oracle.cluster(img, cv, ch, sp.threshold, sp.skip_depth)
        assert np.array_equal(got, want), (sensor, frame)
        checked += 1
    assert checked >= 10
    # the plain per-scan path on one frame per sensor
    ctx = flic.Context(0)
    for sp in specs[:5]:
        d = flic.DeviceScan(torch.from_numpy(frames[sp.sensor][0]).cuda(),
                            torch.from_numpy(tables[sp.sensor][0]).cuda(),
                            torch.from_numpy(tables[sp.sensor][1]).cuda(), sp.threshold, sp.skip_depth)
        ctx.cluster_async(d)
        torch.cuda.synchronize()
        want = oracle.cluster(frames[sp.sensor][0], *tables[sp.sensor], sp.threshold, sp.skip_depth)
        assert np.array_equal(d.labels.cpu().numpy(), want)


@pytest.mark.parametrize("batched,copies", [(True, "kernel"), (False, "kernel"), (True, "dma"), (True, "direct")])
def test_native_served_frames_equal_alone(flic, batched, copies):
    """The library's native serving runtime: every frame's labels (each frame
    with its own pinned label buffer) equal the oracle's for that frame alone."""
    from paper_2003_00575_amd import serve
    specs, frames, tables, rates = serve.make_fleet(10, pool=3, seed=5)
    st, labels = serve.serve_native_once(specs, frames, tables, rates, seconds=0.4, speedup=4.0,
                                         batched=batched, n_streams=3, budget=4 << 30, warmup_s=0.0,
                                         keep_labels=True, copies=copies)
    assert st["frames"] > 20 and st["dropped"] == 0 and st["loop"] == "native"
    if not batched:
        assert st["mean_batch"] == 1.0
    assert len(labels) == st["frames"]
    for (sensor, frame), got in sorted(labels.items()):
        sp = specs[sensor]
        pool = frames[sensor]
        cv, ch = tables[sensor]
        want = oracle.cluster(pool[frame % len(pool)], cv, ch, sp.threshold, sp.skip_depth)
        assert np.array_equal(got, want), (sensor, frame)


def test_native_budget_admission_on_device(flic):
    """The native runtime admits a sensor only while its tables and slots plus
    the context's launch ring fit the budget."""
    from paper_2003_00575_amd import serve
    specs, frames, tables, rates = serve.make_fleet(6, pool=1, seed=2)
    slots = 2
    resident = [sp.skip_depth * (sp.H + sp.W) * 4 + slots * sp.H * sp.W * 8 for sp in specs]
    probe_ctx = flic.Context(0)
    probe = flic.Server(probe_ctx, n_streams=2, max_batch=4, slots_per_sensor=slots)
    for sp in specs[:2]:
        probe.add_sensor(sp.H, sp.W, *tables[sp.sensor], sp.threshold, sp.skip_depth)
    ring = probe_ctx.bytes_in_use()
    probe.close()
    assert ring > 0
    ctx = flic.Context(0)
    srv = flic.Server(ctx, n_streams=2, max_batch=4, slots_per_sensor=slots,
                      hbm_budget=resident[0] + resident[1] + ring)
    for sp in specs[:2]:
        srv.add_sensor(sp.H, sp.W, *tables[sp.sensor], sp.threshold, sp.skip_depth)
    assert ctx.bytes_in_use() == ring
    big = max(specs[2:], key=lambda s: s.H * s.W)
    with pytest.raises(flic.FlicError) as e:
        srv.add_sensor(big.H, big.W, *tables[big.sensor], big.threshold, big.skip_depth)
    assert e.value.status == flic.FLIC_ENOMEM
    srv.close()


def test_budget_admission_on_device(flic):
    from paper_2003_00575_amd import serve
    specs, frames, tables, rates = serve.make_fleet(6, pool=1, seed=2)
    ctx = flic.Context(0)
    be = serve.GpuBackend(ctx, frames, tables, n_streams=2)
    probe = serve.ServingCore(be, 1 << 40, n_streams=2, max_batch=4)
    two = sum(probe.resident_bytes(s) for s in specs[:2])
    biggest = max(specs[:2], key=lambda s: s.H * s.W)
    core = serve.ServingCore(be, two + be.ring_bytes(4, biggest), n_streams=2, max_batch=4)
    core.add_sensor(specs[0])
    core.add_sensor(specs[1])
    with pytest.raises(serve.BudgetError):
        core.add_sensor(specs[2])             # a bigger sensor no longer fits
    assert sorted(core.specs) == [0, 1]
    # what admission charged for the library's launch ring is what it holds
    be.reserve(4)
    assert ctx.bytes_in_use() == core.scratch_reserve()
    assert core.reserved + core.scratch_reserve() <= core.budget


def test_autotune_rules_keep_labels(flic, tmp_path):
    from paper_2003_00575_amd import autotune
    ctx = flic.Context(0)
    shape = (64, 2048, 3)
    timings = autotune.time_shape(ctx, shape, n_scans=4, reps=2)
    assert set(timings) == set(autotune.CANDIDATES) and all(v > 0 for v in timings.values())
    cache = {}
    choice = autotune.record(cache, autotune.gpu_arch(), shape, timings)
    path = str(tmp_path / "tiles.json")
    autotune.save_cache(path, cache)
    again = autotune.load_cache(path)
    assert autotune.apply(ctx, again, autotune.gpu_arch()) == 1
    assert ctx.tile_for(*shape) == choice
    scan = synth.single_scan()
    want = oracle.cluster_scan(scan)
    for tw in autotune.CANDIDATES:
        ctx.set_tile_rule(64, 2048, 3, tw)
        assert ctx.tile_for(64, 2048, 3) == tw
        d = flic.to_device(scan)
        ctx.cluster_async(d)
        torch.cuda.synchronize()
        assert np.array_equal(d.labels.cpu().numpy(), want), tw


@pytest.mark.parametrize("stage", [1, 2])
def test_native_staging_tail_and_pageable_fallback(flic, stage):
    """The native runtime with staging kernels on frames whose size is not a
    multiple of 16 bytes (31 x 1001: the kernel's 4-byte tail) in pinned
    buffers, and on frames in pageable numpy buffers (not device-accessible:
    each falls back to DMA copies); every frame's labels equal the oracle's."""
    shapes = [(31, 1001, 3, 0.6), (16, 1024, 2, 0.4)]
    scans = {s: [synth.synth_scan(H, W, 10.0, -20.0, 12, "iid10", 40 + 10 * s + f, T, N) for f in range(3)]
             for s, (H, W, N, T) in enumerate(shapes)}
    ctx = flic.Context(0)
    srv = flic.Server(ctx, n_streams=2, max_batch=8, slots_per_sensor=2, stage_kernels=stage)
    for s, (H, W, N, T) in enumerate(shapes):
        sc = scans[s][0]
        assert srv.add_sensor(H, W, sc.cos_v, sc.cos_h, T, N) == s
    keep = []
    expect = {}
    tag = 0
    for rep in range(2):
        for s, (H, W, N, T) in enumerate(shapes):
            for f, sc in enumerate(scans[s]):
                if rep == 0:                    # pinned: staged by the kernel
                    src = torch.from_numpy(sc.range_img.copy()).pin_memory()
                    dst = torch.full((H, W), -7, dtype=torch.int32).pin_memory()
                    ptrs = (src.data_ptr(), dst.data_ptr())
                    out = dst
                else:                           # pageable: DMA copies
                    src = np.ascontiguousarray(sc.range_img)
                    dst = np.full((H, W), -7, dtype=np.int32)
                    ptrs = (src.ctypes.data, dst.ctypes.data)
                    out = dst
                keep.append((src, dst))
                now = srv.now()
                srv.submit(now, now, s, ptrs[0], ptrs[1], tag)
                expect[tag] = (out, oracle.cluster(sc.range_img, sc.cos_v, sc.cos_h, T, N))
                tag += 1
                srv.progress(srv.now())
    for _ in range(100000):
        srv.progress(srv.now())
        rec, dropped, launches = srv.records()
        if np.all(np.isfinite(rec["t_done"])):
            break
    torch.cuda.synchronize()
    rec, dropped, launches = srv.records()
    assert dropped == 0 and len(rec) == tag and np.all(np.isfinite(rec["t_done"]))
    for t, (out, want) in expect.items():
        got = out.numpy() if hasattr(out, "numpy") else out
        assert np.array_equal(got, want), t
    srv.close()


def test_native_direct_frames_sharing_buffers(flic):
    """Direct mode (the passes read and write the host buffers) with frames of
    one batch that share their host buffers: a batch's output buffers must not
    overlap any other buffer of it, so the runtime sends such frames through
    their device slots; every frame is served and the labels are right."""
    sc = synth.synth_scan(32, 1800, 10.0, -20.0, 12, "iid10", 77, 0.5, 3)
    ctx = flic.Context(0)
    srv = flic.Server(ctx, n_streams=1, max_batch=8, slots_per_sensor=4, stage_kernels=2)
    sid = srv.add_sensor(32, 1800, sc.cos_v, sc.cos_h, 0.5, 3)
    src = torch.from_numpy(sc.range_img.copy()).pin_memory()
    dst = torch.full((32, 1800), -7, dtype=torch.int32).pin_memory()
    for k in range(4):
        now = srv.now()
        srv.submit(now, now, sid, src.data_ptr(), dst.data_ptr(), k)
    for _ in range(100000):
        srv.progress(srv.now())
        rec, dropped, launches = srv.records()
        if np.all(np.isfinite(rec["t_done"])):
            break
    torch.cuda.synchronize()
    rec, dropped, launches = srv.records()
    assert len(rec) == 4 and dropped == 0 and np.all(np.isfinite(rec["t_done"]))
    assert launches == 1                                   # one batch of all four
    want = oracle.cluster(sc.range_img, sc.cos_v, sc.cos_h, 0.5, 3)
    assert np.array_equal(dst.numpy(), want)
    srv.close()
