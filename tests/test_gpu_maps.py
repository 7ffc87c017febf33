"""The paper's Map Connections (Section III.B.2, map_connections = 1) on the GPU
vs the CPU oracle, bit for bit, through the C ABI: every tile width, ragged
shapes and skip depths 2..8 (maps cross tile columns, tile rows and the
360-degree seam), W not a multiple of the stride, the large batch, a batch
mixing both skip-edge modes and the size threshold, a plan, and the mode
check of plans."""
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


def assert_same(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} labels differ; first at ({r},{c}): "
                             f"gpu {got[r, c]} oracle {want[r, c]}")


def run_gpu(flic, scan, ctx, tile_w=0, m=0):
    ctx.set_tile_width(tile_w)
    d = flic.to_device(scan, min_points=m, map_connections=1)
    d.labels.fill_(-7)
    ctx.cluster_async(d)
    torch.cuda.synchronize()
    ctx.set_tile_width(0)
    return d.labels.cpu().numpy()


@pytest.mark.parametrize("tile_w", [64, 128, 256])
def test_every_tile_width(flic, tile_w):
    ctx = flic.Context(0)
    for scan in (synth.single_scan(), synth.large_batch_scan(3, 0.5), synth.mixed_scan(1)):
        want = oracle.cluster_scan(scan, maps=1)
        assert_same(run_gpu(flic, scan, ctx, tile_w), want, f"tile {tile_w} {scan.H}x{scan.W}")
        # the modes differ on these scenes
        assert not np.array_equal(want, oracle.cluster_scan(scan))


@pytest.mark.parametrize("H, W, N", [(2, 17, 8), (7, 33, 3), (31, 97, 5), (63, 300, 2), (129, 257, 4),
                                     (200, 1000, 3), (300, 70, 6), (128, 4097, 7), (130, 2050, 2)])
def test_random_shapes_ragged(flic, H, W, N):
    ctx = flic.Context(0)
    for seed in range(2):
        scan = synth.random_scan(H, W, N, seed=H * 1000 + W + seed, p_invalid=0.35)
        for tw in (64, 256):
            assert_same(run_gpu(flic, scan, ctx, tw), oracle.cluster_scan(scan, maps=1),
                        f"{H}x{W} N={N} tile {tw} seed {seed}")


def test_large_batch_and_mixed_modes(flic):
    scans = [synth.large_batch_scan(i, (0.3, 0.5, 1.0)[i % 3]) for i in range(32)]
    modes = [(i % 2, (0, 100)[(i // 2) % 2]) for i in range(32)]      # (maps, min_points)
    ctx = flic.Context(0)
    devs = [flic.to_device(s, min_points=m, map_connections=mc) for s, (mc, m) in zip(scans, modes)]
    ctx.cluster_batched(devs)
    torch.cuda.synchronize()
    wants = [oracle.cluster_scan(s, min_points=m, maps=mc) for s, (mc, m) in zip(scans, modes)]
    for i, d in enumerate(devs):
        assert_same(d.labels.cpu().numpy(), wants[i], f"batched scan {i} mode {modes[i]}")
    plan = ctx.plan(devs)
    for d in devs:
        d.labels.fill_(-9)
    plan.launch(devs)
    torch.cuda.synchronize()
    for i, d in enumerate(devs):
        assert_same(d.labels.cpu().numpy(), wants[i], f"plan scan {i}")
    devs[0].map_connections = 1 - devs[0].map_connections
    with pytest.raises(flic.FlicError):
        plan.launch(devs)
    devs[0].map_connections = 2
    with pytest.raises(flic.FlicError):
        ctx.cluster_batched(devs[:1])
    plan.close()


def test_skip_depth_one_is_the_same_in_both_modes(flic):
    ctx = flic.Context(0)
    scan = synth.random_scan(64, 512, 1, seed=5)
    assert_same(run_gpu(flic, scan, ctx), oracle.cluster_scan(scan), "N=1")
