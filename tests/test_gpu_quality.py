"""The quality sweep (Section IV.B metrics on synthetic instances) runs end to
end on the GPU path: labels from the C ABI, scores in range."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_quality_sweep_runs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_00575_amd import quality
    rows = quality._sweep(2, [0.5], [3])
    assert len(rows) == 2
    for r in rows:
        assert r["instances"] > 0
        assert 0.0 < r["iou_mean"] <= 1.0
        assert 0.0 <= r["P_mu"] <= 1.0
