"""GPU labels vs the CPU oracle, bit for bit, through the C ABI.

Covers the per-scan path (stream-ordered and blocking), every tile width,
ragged tiles, skip depths 1..8, the large batch (64 x 128x2048 at three
thresholds), the closed-form stress set, the uneven 256-scan batch (batched
call and hipGraph plan), alone-vs-batch identity, repeated runs (atomic races
would show as run-to-run differences) and degenerate inputs."""
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


def run_gpu(flic, scan, tile_w=None, ctx=None):
    ctx = ctx or flic.Context(0)
    if tile_w is not None:
        ctx.set_tile_width(tile_w)
    d = flic.to_device(scan)
    ctx.cluster_async(d)
    torch.cuda.synchronize()
    if tile_w is not None:
        ctx.set_tile_width(0)
    return d.labels.cpu().numpy()


def assert_same(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        r, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} labels differ; first at ({r},{c}): "
                             f"gpu {got[r, c]} oracle {want[r, c]}")


def test_single_scan_stream_and_blocking(flic):
    scan = synth.single_scan()
    want = oracle.cluster_scan(scan)
    assert_same(run_gpu(flic, scan), want, "async")
    d = flic.to_device(scan)
    out = flic.cluster_sync(d.range_img, d.cos_v, d.cos_h, scan.threshold, scan.skip_depth)
    assert_same(out.cpu().numpy(), want, "blocking")


def test_repeat_runs_identical(flic):
    scan = synth.large_batch_scan(0, 1.0)
    want = oracle.cluster_scan(scan)
    ctx = flic.Context(0)
    d = flic.to_device(scan)
    for i in range(12):
        d.labels.fill_(-7)
        ctx.cluster_async(d)
        torch.cuda.synchronize()
        assert_same(d.labels.cpu().numpy(), want, f"run {i}")


@pytest.mark.parametrize("tile_w", [64, 128, 256])
def test_every_tile_width(flic, tile_w):
    ctx = flic.Context(0)
    for scan in (synth.single_scan(), synth.large_batch_scan(3, 0.5), synth.mixed_scan(1)):
        assert_same(run_gpu(flic, scan, tile_w, ctx), oracle.cluster_scan(scan),
                    f"tile {tile_w} {scan.H}x{scan.W}")


@pytest.mark.parametrize("H, W, N", [(1, 3, 1), (1, 1000, 8), (2, 17, 8), (7, 33, 3), (31, 97, 5),
                                     (63, 300, 2), (129, 257, 4), (200, 1000, 3), (300, 70, 6),
                                     (128, 4096, 8), (5, 4097, 1)])
def test_random_shapes_ragged(flic, H, W, N):
    ctx = flic.Context(0)
    for seed in range(3):
        scan = synth.random_scan(H, W, N, seed=seed, threshold=0.45, p_invalid=0.25)
        want = oracle.cluster_scan(scan)
        for tw in (64, 128, 256):
            assert_same(run_gpu(flic, scan, tw, ctx), want, f"{H}x{W} N={N} tile {tw} seed {seed}")


def test_degenerate_inputs(flic):
    ctx = flic.Context(0)
    H, W, N = 40, 300, 3
    base = synth.random_scan(H, W, N, seed=5)
    cases = {}
    s = synth.random_scan(H, W, N, seed=5); s.range_img[:] = 0.0; cases["all missing"] = s
    s = synth.random_scan(H, W, N, seed=5, p_invalid=0.0); s.threshold = 1e30; cases["huge T"] = s
    s = synth.random_scan(H, W, N, seed=5); s.threshold = 0.0; cases["T=0"] = s
    s = synth.random_scan(H, W, N, seed=5)
    flat = s.range_img.reshape(-1)
    flat[::7] = np.nan; flat[1::7] = np.inf; flat[2::7] = -np.inf; flat[3::7] = -0.0
    flat[4::7] = -1.0; flat[5::11] = np.float32(1e-42)
    cases["special floats"] = s
    s = synth.random_scan(H, W, N, seed=5); s.range_img[:] = 3.0; s.threshold = 0.0
    s.cos_v[:] = 1.0; s.cos_h[:] = 1.0; cases["coincident points at T=0"] = s
    s = synth.random_scan(H, W, N, seed=5); s.range_img *= np.float32(1e-20); s.threshold = 1e-20
    cases["subnormal distances"] = s
    s = synth.random_scan(H, W, N, seed=5); s.range_img *= np.float32(1e19); s.threshold = 1e19
    cases["overflowing squares"] = s
    s = synth.random_scan(H, W, N, seed=5); s.cos_h[:, ::3] = np.nan; s.cos_v[:, ::5] = np.inf
    cases["non-finite tables"] = s
    assert base is not None
    for name, scan in cases.items():
        assert_same(run_gpu(flic, scan, None, ctx), oracle.cluster_scan(scan), name)


@pytest.mark.parametrize("T", [0.3, 0.5, 1.0])
def test_stress_set_closed_form(flic, T):
    """Serpentines spanning every tile border, checkerboard, wrap-seam runs,
    all-valid; expected labels known in closed form (and equal to the oracle)."""
    H, W = 64, 4096
    rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    ctx = flic.Context(0)
    scans = []
    for N in range(1, 6):
        for name in synth.STRESS_PATTERNS:
            scan = synth.stress_scan(name, T, N, seed=N)
            v = (scan.range_img > 0)
            if name in ("serpentine_rows", "serpentine_cols", "all_valid"):
                exp = np.where(v, 0, -1)
            elif name == "checkerboard":
                exp = np.where(v, rr * W + cc if N == 1 else np.where(rr % 2 == 0, 0, W + 1), -1)
            else:
                exp = np.where(v, rr * W, -1)
            scans.append((scan, exp, f"{name} N={N}"))
    for tw in (64, 128, 256):
        for scan, exp, what in scans:
            assert_same(run_gpu(flic, scan, tw, ctx), exp, f"{what} tile {tw}")
    # the same set as one batched launch
    devs = [flic.to_device(s) for s, _, _ in scans]
    ctx.cluster_batched(devs)
    torch.cuda.synchronize()
    for d, (scan, exp, what) in zip(devs, scans):
        assert_same(d.labels.cpu().numpy(), exp, f"batched {what}")


@pytest.mark.parametrize("T", [0.3, 0.5, 1.0])
def test_large_batch_64x128x2048(flic, T):
    scans = [synth.large_batch_scan(i, T) for i in range(64)]
    devs = [flic.to_device(s) for s in scans]
    ctx = flic.Context(0)
    ctx.cluster_batched(devs)
    torch.cuda.synchronize()
    for i, (s, d) in enumerate(zip(scans, devs)):
        assert_same(d.labels.cpu().numpy(), oracle.cluster_scan(s), f"scan {i} T={T}")


def test_uneven_batch_batched_plan_and_alone(flic):
    scans = [synth.mixed_scan(i) for i in range(256)]
    want = [oracle.cluster_scan(s) for s in scans]
    ctx = flic.Context(0)
    devs = [flic.to_device(s) for s in scans]
    ctx.cluster_batched(devs)
    torch.cuda.synchronize()
    for i, d in enumerate(devs):
        assert_same(d.labels.cpu().numpy(), want[i], f"batched scan {i}")
    # hipGraph plan, launched several times with fresh outputs
    plan = ctx.plan(devs)
    for rep in range(3):
        for d in devs:
            d.labels.fill_(-9)
        plan.launch(devs)
        torch.cuda.synchronize()
        for i, d in enumerate(devs):
            assert_same(d.labels.cpu().numpy(), want[i], f"plan rep {rep} scan {i}")
    # new output buffers and thresholds through the same plan
    devs2 = [flic.DeviceScan(d.range_img, d.cos_v, d.cos_h, 0.8, d.skip_depth) for d in devs]
    plan.launch(devs2)
    torch.cuda.synchronize()
    for i in range(0, 256, 17):
        s = scans[i]
        exp = oracle.cluster(s.range_img, s.cos_v, s.cos_h, 0.8, s.skip_depth)
        assert_same(devs2[i].labels.cpu().numpy(), exp, f"replanned scan {i}")
    plan.close()
    # alone
    for i in range(0, 256, 5):
        assert_same(run_gpu(flic, scans[i], None, ctx), want[i], f"alone scan {i}")


def test_batched_mixed_skip_depths_and_stream(flic):
    scans = [synth.random_scan(37 + 9 * i, 300 + 101 * i, 1 + i % 8, seed=i) for i in range(16)]
    ctx = flic.Context(0)
    devs = [flic.to_device(s) for s in scans]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx.cluster_batched(devs, stream=st)
    st.synchronize()
    for i, (s, d) in enumerate(zip(scans, devs)):
        assert_same(d.labels.cpu().numpy(), oracle.cluster_scan(s), f"scan {i}")


def _border_pairs_scan(H=128, W=16384, N=3, seg=4, tile_w=64):
    """Every even row holds a short segment across every tile-column border
    (and the 360-degree seam), each row at its own range 1 m from the next, so
    no vertical or skip edge joins two rows: about (H/2) * (W/tile_w) distinct
    pairs of tile roots (16384) are joined by the border pass, every border
    item holding many independent joins."""
    img = np.zeros((H, W), np.float32)
    for r in range(0, H, 2):
        for b in range(0, W, tile_w):
            cols = np.arange(b - seg, b + seg) % W
            img[r, cols] = 10.0 + r
    phi = synth.elevations(H, 2.0, -24.8)
    cos_v, cos_h = synth.make_tables(phi, W, N)
    return synth.Scan(img, cos_v, cos_h, 0.5, N, None, 0)


def test_many_border_components(flic):
    scan = _border_pairs_scan()
    want = oracle.cluster_scan(scan)
    # every segment is one component spanning two tiles
    assert len(np.unique(want[want >= 0])) == (scan.range_img.shape[0] // 2) * (scan.range_img.shape[1] // 64)
    assert_same(run_gpu(flic, scan, tile_w=64), want, "many border components")
    ctx = flic.Context(0)
    ctx.set_tile_width(64)
    d = flic.to_device(scan)
    plan = ctx.plan([d])
    plan.relaunch()
    torch.cuda.synchronize()
    assert_same(d.labels.cpu().numpy(), want, "many border components, plan")
    plan.close()


def test_plan_relaunch_on_two_streams(flic):
    """A plan's launches share its scratch: back-to-back launches of an
    unchanged plan on two streams must run one after the other, so every
    launch writes the oracle's labels."""
    scans = [synth.large_batch_scan(i, 0.5) for i in range(8)]
    want = [oracle.cluster_scan(s) for s in scans]
    ctx = flic.Context(0)
    devs = [flic.to_device(s) for s in scans]
    plan = ctx.plan(devs)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(6):
        for d in devs:
            d.labels.fill_(-9)
        torch.cuda.synchronize()
        for k in range(8):
            plan.relaunch(streams[k % 2])
        torch.cuda.synchronize()
        for i, d in enumerate(devs):
            assert_same(d.labels.cpu().numpy(), want[i], f"rep {rep} scan {i}")
    plan.close()


@pytest.mark.parametrize("parts", [2, 3, 7])
def test_plan_parts_as_parallel_branches(flic, parts):
    """A plan whose launch groups are split into parallel graph branches
    gives the same labels as the oracle (mixed shapes, relaunched)."""
    scans = [synth.mixed_scan(i) for i in range(0, 40)]
    want = [oracle.cluster_scan(s) for s in scans]
    ctx = flic.Context(0)
    ctx.set_plan_parts(parts)
    devs = [flic.to_device(s) for s in scans]
    plan = ctx.plan(devs)
    for rep in range(2):
        for d in devs:
            d.labels.fill_(-9)
        plan.relaunch()
        torch.cuda.synchronize()
        for i, d in enumerate(devs):
            assert_same(d.labels.cpu().numpy(), want[i], f"parts {parts} rep {rep} scan {i}")
    plan.close()


def test_batched_host_copies_in_and_out(flic):
    """flic_cluster_batched_host: ranges copied in from pinned host buffers,
    the batch clustered, labels copied out to pinned host buffers, all on one
    stream; equal to the oracle (mixed shapes), twice on the same buffers with
    new host data."""
    import ctypes
    ctx = flic.Context(0)
    stream = torch.cuda.Stream()
    for rep in range(2):
        scans = [synth.mixed_scan(40 * rep + i) for i in range(10)]
        devs = [flic.to_device(s) for s in scans]
        for d in devs:
            d.range_img.zero_()                   # the data must come from the host copy
        h_in = [torch.from_numpy(s.range_img).pin_memory() for s in scans]
        h_out = [torch.full(s.range_img.shape, -7, dtype=torch.int32).pin_memory() for s in scans]
        arr = flic.Context.scan_array(devs)
        n = len(devs)
        hin = (ctypes.c_void_p * n)(*[t.data_ptr() for t in h_in])
        hout = (ctypes.c_void_p * n)(*[t.data_ptr() for t in h_out])
        ctx.cluster_batched_host(arr, n, hin, hout, stream)
        stream.synchronize()
        for i, s in enumerate(scans):
            assert_same(h_out[i].numpy(), oracle.cluster_scan(s), f"rep {rep} scan {i}")
