"""Instance-quality metrics of Section IV.B (Eq. 5 Jaccard index, Eq. 6
precision over overlap bins): hand-derived cases, the under-segmentation rule,
the 100-point instance filter, missing pixels, and a set-based brute force."""
import numpy as np
import pytest

from paper_2003_00575_amd import quality


def _arr(*parts):
    return np.concatenate([np.full(n, v, dtype=np.int64) for v, n in parts])


def test_identical_segmentation_is_perfect():
    gt = _arr((1, 150), (2, 300), (0, 50), (-1, 10))
    lab = _arr((7, 150), (3, 300), (-1, 60))
    ious = quality.instance_ious(lab, gt, np.ones(gt.size, bool))
    assert ious == {1: 1.0, 2: 1.0}
    s = quality.summarize(ious.values())
    assert s["iou_mean"] == 1.0 and s["P_mu"] == 1.0 and s["P_0.95"] == 1.0


def test_hand_example_partial_overlap():
    # instance 1: 120 points; cluster 5 holds 100 of them and 40 other points
    gt = _arr((1, 100), (1, 20), (0, 40))
    lab = _arr((5, 100), (-1, 20), (5, 40))
    ious = quality.instance_ious(lab, gt, np.ones(gt.size, bool))
    assert ious[1] == pytest.approx(100 / 160)
    s = quality.summarize(ious.values())
    assert s["P_0.60"] == 1.0 and s["P_0.65"] == 0.0


def test_hand_example_bins_exact():
    # J = 0.625 passes the bins 0.50, 0.55 and 0.60 only
    gt = _arr((1, 100), (1, 20), (0, 40))
    lab = _arr((5, 100), (-1, 20), (5, 40))
    s = quality.summarize(quality.instance_ious(lab, gt, np.ones(gt.size, bool)).values())
    assert [s[f"P_{x:.2f}"] for x in quality.BINS] == [1, 1, 1, 0, 0, 0, 0, 0, 0, 0]
    assert s["P_mu"] == pytest.approx(0.3)


def test_under_segmentation_keeps_the_better_instance():
    # instances 1 (150) and 2 (120) in one cluster of 270: J = 150/270 and 120/270
    gt = _arr((1, 150), (2, 120))
    lab = _arr((9, 270))
    ious = quality.instance_ious(lab, gt, np.ones(gt.size, bool))
    assert ious[1] == pytest.approx(150 / 270)
    assert ious[2] == 0.0


def test_small_instances_and_missing_pixels():
    gt = _arr((1, 99), (2, 100), (3, 130))
    lab = _arr((4, 99), (5, 100), (6, 130))
    measured = np.ones(gt.size, bool)
    measured[-40:] = False                          # instance 3 drops to 90 measured points
    ious = quality.instance_ious(lab, gt, measured)
    assert set(ious) == {2}
    # an instance whose points are all unlabelled is not found
    lab2 = lab.copy()
    lab2[99:199] = -1
    assert quality.instance_ious(lab2, gt, np.ones(gt.size, bool))[2] == 0.0


def _brute(lab, gt, measured, min_points=100):
    pts = [i for i in range(len(gt)) if measured[i]]
    inst = {}
    for i in pts:
        if gt[i] > 0:
            inst.setdefault(gt[i], set()).add(i)
    clusters = {}
    for i in pts:
        if lab[i] >= 0:
            clusters.setdefault(lab[i], set()).add(i)
    best = {}
    for g, A in inst.items():
        if len(A) < min_points:
            continue
        cands = [(len(A & B), -c, c) for c, B in clusters.items() if A & B]
        if not cands:
            best[g] = (None, 0.0)
            continue
        _, _, c = max(cands)
        B = clusters[c]
        best[g] = (c, len(A & B) / len(A | B))
    out = {}
    for g, (c, j) in best.items():
        keep = c is not None and all(j > j2 or (j == j2 and g < g2)
                                     for g2, (c2, j2) in best.items() if c2 == c and g2 != g)
        out[g] = j if keep else 0.0
    return out


@pytest.mark.parametrize("seed", range(5))
def test_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 2000
    gt = rng.integers(-1, 6, size=n)
    # clusters: mostly follow gt, with noise and merges
    lab = np.where(rng.uniform(size=n) < 0.8, gt % 4, rng.integers(-1, 8, size=n))
    measured = rng.uniform(size=n) < 0.9
    got = quality.instance_ious(lab, gt, measured)
    want = _brute(lab, gt, measured)
    assert set(got) == set(want)
    for g in want:
        assert got[g] == pytest.approx(want[g]), g


def test_literal_first_channel_rule_keeps_cells_below_missing_ones():
    """Under the literal reading only row 0 borrows the pair below; a cell of a
    lower row whose upper neighbour is missing computes Eq. (2) with d1 = 0,
    tan(beta) = -tan(alpha) < 0, and stays (hand-derived 3 x 3 case)."""
    from paper_2003_00575_amd.quality import literal_first_channel
    r = np.array([[0.0, 2.0, 2.0],
                  [3.0, 0.0, 3.0],
                  [4.0, 4.0, np.nan]], np.float32)
    ext = np.array([[0, 1, 1],
                    [1, 0, 1],
                    [1, 1, 0]], bool)
    want = np.array([[0, 1, 1],      # row 0: the first-channel rule, as extended
                     [0, 0, 1],      # (1,0) lies under a missing cell: kept
                     [1, 0, 0]], bool)   # (2,1) lies under a missing cell: kept
    assert np.array_equal(literal_first_channel(r, ext), want)
