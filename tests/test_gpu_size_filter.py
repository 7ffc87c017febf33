"""Cluster-size threshold (Section III.B.1) on the GPU vs the CPU oracle, bit
for bit, through the C ABI: the counting kernels at every tile width, ragged
shapes, the hand-derived example, mixed batches (scans with and without a
threshold), the full 64 x 128x2048 batch at the paper's 100 points, plans
whose min_points change between launches, thousands of two-tile components,
repeated runs, and the degenerate thresholds."""
import numpy as np
import pytest

import oracle
from helpers import read_golden
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


def assert_same(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} labels differ; first at ({r},{c}): "
                             f"gpu {got[r, c]} oracle {want[r, c]}")


def run_gpu(flic, scan, m, ctx, tile_w=0):
    ctx.set_tile_width(tile_w)
    d = flic.to_device(scan, min_points=m)
    d.labels.fill_(-7)
    ctx.cluster_async(d)
    torch.cuda.synchronize()
    ctx.set_tile_width(0)
    return d.labels.cpu().numpy()


def test_golden_example(flic):
    g = read_golden("size_filter_5x8.txt")
    H, W = int(g["H"]), int(g["W"])
    scan = synth.Scan(g["range"].astype(np.float32), np.ones((1, H), np.float32),
                      np.ones((1, W), np.float32), float(g["T"]), 1, None, 0)
    ctx = flic.Context(0)
    for m, key in [(1, "labels_m0"), (2, "labels_m2"), (3, "labels_m3"), (6, "labels_m4")]:
        assert_same(run_gpu(flic, scan, m, ctx), g[key].astype(np.int32), f"golden m={m}")
    assert (run_gpu(flic, scan, 7, ctx) == -1).all()


@pytest.mark.parametrize("tile_w", [64, 128, 256])
def test_every_tile_width(flic, tile_w):
    ctx = flic.Context(0)
    for scan in (synth.single_scan(), synth.large_batch_scan(3, 0.5), synth.mixed_scan(1)):
        lab = oracle.cluster_scan(scan)
        for m in (1, 2, 10, 100):
            assert_same(run_gpu(flic, scan, m, ctx, tile_w), oracle.filter_small(lab, m),
                        f"tile {tile_w} {scan.H}x{scan.W} m={m}")


@pytest.mark.parametrize("H, W, N", [(1, 3, 1), (2, 17, 8), (7, 33, 3), (31, 97, 5), (63, 300, 2),
                                     (129, 257, 4), (200, 1000, 3), (300, 70, 6), (128, 4096, 8)])
def test_random_shapes_ragged(flic, H, W, N):
    ctx = flic.Context(0)
    scan = synth.random_scan(H, W, N, seed=H * 1000 + W)
    lab = oracle.cluster_scan(scan)
    for m in (3, 50):
        assert_same(run_gpu(flic, scan, m, ctx), oracle.filter_small(lab, m), f"{H}x{W} N={N} m={m}")


def test_degenerate_thresholds(flic):
    ctx = flic.Context(0)
    scan = synth.large_batch_scan(5, 0.5)
    lab = oracle.cluster_scan(scan)
    # 1 keeps everything (the counting kernels leave the labels alone)
    assert_same(run_gpu(flic, scan, 1, ctx), lab, "m=1")
    # more than the image: nothing survives
    assert (run_gpu(flic, scan, scan.range_img.size + 1, ctx) == -1).all()
    # an all-missing image
    empty = synth.Scan(np.zeros_like(scan.range_img), scan.cos_v, scan.cos_h, 0.5, scan.skip_depth, None, 0)
    assert (run_gpu(flic, empty, 100, ctx) == -1).all()
    # a single component covering the whole image: exactly H*W points
    full = synth.Scan(np.full_like(scan.range_img, 10.0), scan.cos_v, scan.cos_h, 0.5, scan.skip_depth,
                      None, 0)
    P = full.range_img.size
    assert (oracle.cluster_scan(full) == 0).all()
    assert (run_gpu(flic, full, P, ctx) == 0).all()
    assert (run_gpu(flic, full, P + 1, ctx) == -1).all()


def test_negative_min_points_rejected(flic):
    ctx = flic.Context(0)
    d = flic.to_device(synth.single_scan(), min_points=-1)
    d.labels.fill_(-7)
    with pytest.raises(flic.FlicError):
        ctx.cluster_batched([d])
    torch.cuda.synchronize()
    assert (d.labels == -7).all()


def test_repeat_runs_identical(flic):
    scan = synth.large_batch_scan(0, 1.0)
    want = oracle.cluster_scan(scan, min_points=100)
    ctx = flic.Context(0)
    d = flic.to_device(scan, min_points=100)
    for i in range(8):
        d.labels.fill_(-7)
        ctx.cluster_async(d)
        torch.cuda.synchronize()
        assert_same(d.labels.cpu().numpy(), want, f"run {i}")


def test_large_batch_64x128x2048_paper_threshold(flic):
    scans = [synth.large_batch_scan(i, 0.5) for i in range(64)]
    devs = [flic.to_device(s, min_points=100) for s in scans]
    ctx = flic.Context(0)
    ctx.cluster_batched(devs)
    torch.cuda.synchronize()
    for i, (s, d) in enumerate(zip(scans, devs)):
        assert_same(d.labels.cpu().numpy(), oracle.cluster_scan(s, min_points=100), f"scan {i}")


def test_mixed_batch_and_plan(flic):
    scans = [synth.mixed_scan(i) for i in range(48)]
    ms = [(0, 1, 5, 100)[i % 4] for i in range(48)]
    labs = [oracle.cluster_scan(s) for s in scans]
    ctx = flic.Context(0)
    devs = [flic.to_device(s, min_points=m) for s, m in zip(scans, ms)]
    ctx.cluster_batched(devs)
    torch.cuda.synchronize()
    for i, d in enumerate(devs):
        assert_same(d.labels.cpu().numpy(), oracle.filter_small(labs[i], ms[i]), f"batched scan {i}")
    plan = ctx.plan(devs)
    for rep in range(2):
        for d in devs:
            d.labels.fill_(-9)
        plan.launch(devs)
        torch.cuda.synchronize()
        for i, d in enumerate(devs):
            assert_same(d.labels.cpu().numpy(), oracle.filter_small(labs[i], ms[i]), f"plan {rep} scan {i}")
    # other positive thresholds through the same plan (descriptor refresh)
    ms2 = [0 if m == 0 else (7 if m != 7 else 3) for m in ms]
    for d, m in zip(devs, ms2):
        d.min_points = m
    plan.launch(devs)
    torch.cuda.synchronize()
    for i, d in enumerate(devs):
        assert_same(d.labels.cpu().numpy(), oracle.filter_small(labs[i], ms2[i]), f"replanned scan {i}")
    # a threshold switched on or off does not match the plan
    devs[0].min_points = 5
    with pytest.raises(flic.FlicError):
        plan.launch(devs)
    devs[0].min_points = 0
    devs[1].min_points = 0
    with pytest.raises(flic.FlicError):
        plan.launch(devs)
    plan.close()


def _border_pairs_scan(H=128, W=16384, N=3, seg=4, tile_w=64):
    """Every even row holds a 2*seg-pixel segment across every tile-column
    border (and the 360-degree seam), each row at its own range, so about
    (H/2) * (W/tile_w) components of exactly 2*seg pixels, seg in each of two
    tiles, whose two halves' counts the border passes must sum."""
    img = np.zeros((H, W), np.float32)
    for r in range(0, H, 2):
        for b in range(0, W, tile_w):
            cols = np.arange(b - seg, b + seg) % W
            img[r, cols] = 10.0 + r
    phi = synth.elevations(H, 2.0, -24.8)
    cos_v, cos_h = synth.make_tables(phi, W, N)
    return synth.Scan(img, cos_v, cos_h, 0.5, N, None, 0)


def test_border_components_sum_counts(flic):
    scan = _border_pairs_scan()
    lab = oracle.cluster_scan(scan)
    ctx = flic.Context(0)
    for m in (5, 8, 9):        # each half has 4 pixels; only the summed 8 reaches 5 and 8
        want = oracle.filter_small(lab, m)
        assert (want >= 0).any() == (m <= 8)
        assert_same(run_gpu(flic, scan, m, ctx, tile_w=64), want, f"border components m={m}")
