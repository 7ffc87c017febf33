"""flic_cluster_noalloc (the allocation-free entry point: scratch from the
library's fixed device array) against flic_cluster_async (the same kernels on
a context's allocated scratch), through the C ABI: two calls in a row, the
second on a smaller scan, bit for bit; plus the size limit, rejected on the
host before any HIP call."""
import numpy as np
import pytest

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


def _with_context(flic, scan):
    d = flic.to_device(scan)
    flic.Context(0).cluster_async(d)
    torch.cuda.synchronize()
    return d.labels.cpu().numpy()


def _noalloc(flic, scan, stream=None):
    d = flic.to_device(scan)
    d.labels.fill_(-7)
    out = flic.cluster_noalloc(d.range_img, d.cos_v, d.cos_h, scan.threshold, scan.skip_depth,
                               out=d.labels, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_allocating_entry_point_twice(flic):
    big = synth.large_batch_scan(3, 0.5)                 # 128 x 2048, skip 3
    small = synth.single_scan(1)                         # 64 x 2048: a smaller second call
    for scan in (big, small):
        want = _with_context(flic, scan)
        got = _noalloc(flic, scan)
        assert np.array_equal(got, want), f"{scan.range_img.shape}: {(got != want).sum()} labels differ"


def test_noalloc_ragged_shapes_and_side_stream(flic):
    st = torch.cuda.Stream()
    for i, (H, W, N) in enumerate([(300, 70, 3), (5, 4097, 8), (128, 4096, 8), (1, 3, 1)]):
        scan = synth.random_scan(H, W, N, seed=40 + i)
        want = _with_context(flic, scan)
        got = _noalloc(flic, scan, stream=st)
        assert np.array_equal(got, want), f"{H}x{W} N={N}: {(got != want).sum()} labels differ"


def test_noalloc_rejects_scans_beyond_its_scratch(flic):
    # 1024 x 4096 needs a 16 MiB parent array alone: refused before any launch
    R, LBL, CV, CH = 0x10000000, 0x20000000, 0x30000000, 0x40000000
    assert flic.cluster_noalloc_raw(R, 1024, 4096, CV, CH, 0.5, 3, LBL, 0) == flic.FLIC_EINVAL
    assert "scratch" in flic.last_error()
