"""Pins of the oracle's paper-literal Map Connections (Section III.B.2): a map
of stride k holds the points whose row and column are multiples of k and joins
each with its k-th neighbour right (with wrap) and below.  Checked against an
all-pairs brute force with explicit points, a library CCL over lattice edge
lists, the nesting of the edge sets (direct edges within maps within dense
skips), and a hand-built gap that only a map point can bridge."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2003_00575_amd import synth
from helpers import (U32, UnionFind, canonical, canonical_fast, explicit_points_distance,
                     is_measurement, neighbour_pairs)


def _brute_force_maps(scan):
    """Explicit-point float64 distances over every neighbour pair whose first
    end lies on the pair's map (k = 1: every pixel), joined by union-find;
    None when a pair lies within the float32 margin of the threshold."""
    H, W, N = scan.H, scan.W, scan.skip_depth
    r = scan.range_img.reshape(-1)
    T2 = float(np.float32(scan.threshold) * np.float32(scan.threshold))
    uf = UnionFind(H * W)
    for p, q, kind, k in neighbour_pairs(H, W, N):
        rp, cp = divmod(p, W)
        if k >= 2 and not (rp % k == 0 and cp % k == 0):
            continue
        if not (is_measurement(r[p]) and is_measurement(r[q])):
            continue
        cs = scan.cos_v[k - 1, rp] if kind == "v" else scan.cos_h[k - 1, cp]
        a, b = float(r[p]), float(r[q])
        d = explicit_points_distance(a, b, float(cs))
        if abs(d * d - T2) <= 8 * U32 * (a * a + b * b) + 8 * U32 * T2:
            return None
        if d * d <= T2:
            uf.union(p, q)
    lab = np.array([uf.find(i) if is_measurement(r[i]) else -1 for i in range(H * W)])
    return canonical(lab.reshape(H, W))


@pytest.mark.parametrize("H, W, N", [(2, 5, 2), (4, 9, 2), (5, 12, 3), (6, 11, 4), (4, 17, 8)])
def test_brute_force_tiny(H, W, N):
    checked, seed = 0, 0
    while checked < 10 and seed < 400:
        seed += 1
        scan = synth.random_scan(H, W, N, seed=2000 * H + seed, threshold=0.45,
                                 p_invalid=0.3, spread=0.35)
        bf = _brute_force_maps(scan)
        if bf is None:
            continue
        np.testing.assert_array_equal(oracle.cluster_scan(scan, maps=1), bf)
        checked += 1
    assert checked >= 10


def _csgraph_maps(scan):
    """Lattice edge lists from numpy shifted copies (float32 ufuncs, Eq. 4)."""
    H, W, N = scan.H, scan.W, scan.skip_depth
    img = scan.range_img
    valid = is_measurement(img)
    val = np.where(valid, img, np.float32(np.nan)).astype(np.float32)
    t2 = np.float32(scan.threshold) * np.float32(scan.threshold)
    idx = np.arange(H * W).reshape(H, W)
    rows, cols = np.indices((H, W))
    us, vs = [], []
    for k in range(1, N + 1):
        lat = np.ones((H, W), bool) if k == 1 else (rows % k == 0) & (cols % k == 0)
        if k < H:
            a, b = val[:-k], val[k:]
            c2 = (np.float32(2) * scan.cos_v[k - 1, : H - k])[:, None]
            d2 = (a * a + b * b) - c2 * (a * b)
            e = (d2 <= t2) & lat[:-k]
            us.append(idx[:-k][e]); vs.append(idx[k:][e])
        a, b = val, np.roll(val, -k, axis=1)
        c2 = (np.float32(2) * scan.cos_h[k - 1])[None, :]
        d2 = (a * a + b * b) - c2 * (a * b)
        e = (d2 <= t2) & lat
        us.append(idx[e]); vs.append(np.roll(idx, -k, axis=1)[e])
    u = np.concatenate(us); v = np.concatenate(vs)
    g = coo_matrix((np.ones(u.size), (u, v)), shape=(H * W, H * W))
    _, comp = connected_components(g, directed=False)
    return canonical_fast(np.where(valid.reshape(-1), comp, -1).reshape(H, W))


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_csgraph_lattice_edges(N):
    with np.errstate(invalid="ignore"):
        for seed in range(3):
            scan = synth.random_scan(24, 64, N, seed=300 + seed, threshold=0.4, p_invalid=0.3)
            np.testing.assert_array_equal(oracle.cluster_scan(scan, maps=1), _csgraph_maps(scan))


def _refines(fine, coarse):
    """Every component of `fine` lies inside one component of `coarse`."""
    f, c = fine.reshape(-1), coarse.reshape(-1)
    m = f >= 0
    pairs = np.unique(np.stack([f[m], c[m]]), axis=1)
    return np.unique(pairs[0]).size == pairs.shape[1]


def test_nesting_direct_maps_dense():
    for seed in range(4):
        scan = synth.random_scan(32, 128, 4, seed=50 + seed, threshold=0.5, p_invalid=0.35)
        direct = oracle.cluster(scan.range_img, scan.cos_v[:1], scan.cos_h[:1], scan.threshold, 1)
        maps = oracle.cluster_scan(scan, maps=1)
        dense = oracle.cluster_scan(scan)
        assert _refines(direct, maps) and _refines(maps, dense)
    # N = 1 has no skip edges: both modes agree
    scan = synth.random_scan(16, 40, 1, seed=7)
    np.testing.assert_array_equal(oracle.cluster_scan(scan, maps=1), oracle.cluster_scan(scan))


def test_gap_bridged_only_on_the_map():
    """A missing column 5 splits a flat object; at N = 2 the stride-2 map
    bridges it only from even rows and even columns: with column 4 on the map
    the halves join, with the gap shifted to column 6 (bridge from column 5,
    off the map) they stay apart."""
    H, W = 4, 16
    cv = np.ones((2, H), np.float32)
    ch = np.ones((2, W), np.float32)
    img = np.full((H, W), 5.0, np.float32)
    img[:, 12:] = 0.0
    img[:, 5] = 0.0
    lab = oracle.cluster(img, cv, ch, 0.5, 2, maps=1)
    assert lab[0, 0] == lab[0, 6]
    img2 = np.full((H, W), 5.0, np.float32)
    img2[:, 12:] = 0.0
    img2[:, 6] = 0.0
    lab2 = oracle.cluster(img2, cv, ch, 0.5, 2, maps=1)
    assert lab2[0, 0] != lab2[0, 7]
    dense2 = oracle.cluster(img2, cv, ch, 0.5, 2)
    assert dense2[0, 0] == dense2[0, 7]
