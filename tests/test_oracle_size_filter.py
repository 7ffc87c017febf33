"""Pins of the oracle's cluster-size threshold (Section III.B.1: clusters with
fewer than a minimum number of measurements are no cluster candidates) against
a hand-derived worked example, a pairwise brute force on tiny inputs and
invariants of the definition."""
import numpy as np
import pytest

import oracle
from paper_2003_00575_amd import synth
from helpers import read_golden


def _golden():
    g = read_golden("size_filter_5x8.txt")
    H, W = int(g["H"]), int(g["W"])
    r = g["range"].astype(np.float32)
    ones_v = np.ones((1, H), dtype=np.float32)
    ones_h = np.ones((1, W), dtype=np.float32)
    return g, r, ones_v, ones_h, float(g["T"])


@pytest.mark.parametrize("m, key", [(0, "labels_m0"), (1, "labels_m0"), (2, "labels_m2"),
                                    (3, "labels_m3"), (4, "labels_m4"), (5, "labels_m4"),
                                    (6, "labels_m4"), (7, None), (100, None)])
def test_golden_size_filter(m, key):
    g, r, cv, chh, T = _golden()
    got = oracle.cluster(r, cv, chh, T, 1, min_points=m)
    want = g[key].astype(np.int32) if key else np.full(r.shape, -1, np.int32)
    np.testing.assert_array_equal(got, want)


def _brute_filter(labels, m):
    """Pairwise count: pixel p survives iff at least m pixels share its label."""
    flat = labels.ravel().tolist()
    out = []
    for lp in flat:
        if lp < 0:
            out.append(-1)
            continue
        n = 0
        for lq in flat:
            if lq == lp:
                n += 1
        out.append(lp if n >= m else -1)
    return np.array(out, dtype=np.int32).reshape(labels.shape)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 6)), int(rng.integers(3, 9))
    scan = synth.random_scan(H, W, 1, seed, threshold=0.5, p_invalid=0.3)
    lab = oracle.cluster_scan(scan)
    for m in range(0, 8):
        np.testing.assert_array_equal(oracle.filter_small(lab, m), _brute_filter(lab, m))


def test_brute_force_arbitrary_label_values():
    # the filter needs no canonical labels: any ids in [0, H*W) are counted
    rng = np.random.default_rng(7)
    lab = rng.integers(-1, 6, size=(4, 5)).astype(np.int32)
    for m in range(0, 10):
        np.testing.assert_array_equal(oracle.filter_small(lab, m), _brute_filter(lab, m))


def test_invariants_on_synthetic_scan():
    scan = synth.single_scan(seed=3)
    lab = oracle.cluster_scan(scan)
    P = lab.size
    np.testing.assert_array_equal(oracle.filter_small(lab, 0), lab)
    np.testing.assert_array_equal(oracle.filter_small(lab, 1), lab)
    assert (oracle.filter_small(lab, P + 1) == -1).all()
    prev = lab
    for m in (2, 5, 20, 100, 400):
        cur = oracle.filter_small(lab, m)
        kept = cur >= 0
        # kept pixels keep their label; the kept set shrinks as m grows
        np.testing.assert_array_equal(cur[kept], lab[kept])
        assert not (kept & ~(prev >= 0)).any()
        # idempotent, and what m removes is exactly what the labels of size < m cover
        np.testing.assert_array_equal(oracle.filter_small(cur, m), cur)
        prev = cur
    # the paper's value (100) removes something and keeps something on this scene
    f100 = oracle.filter_small(lab, 100)
    assert (f100 >= 0).any() and ((lab >= 0) & (f100 < 0)).any()


def test_filter_argument_errors():
    lab = np.zeros((2, 3), dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.filter_small(lab, -1)
    bad = lab.copy()
    bad[0, 0] = 6                          # outside [0, H*W)
    with pytest.raises(ValueError):
        oracle.filter_small(bad, 2)
    bad[0, 0] = -2
    with pytest.raises(ValueError):
        oracle.filter_small(bad, 2)
