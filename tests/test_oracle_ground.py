"""Pins of the oracle's ground extraction (Section III.A, Eq. 1/2, the height
image and the first-channel rule) against geometry that does not come from the
oracle: noise-free raycast ground planes, vertical surfaces, tilted planes whose
slope is set by explicit 2-D points, the height line, and the handling of
missing cells."""
import math

import numpy as np
import pytest

import oracle
from paper_2003_00575_amd import synth


def _flat_ground(H, W, top, bottom):
    phi = synth.elevations(H, top, bottom)
    t, _ = synth.raycast(phi, W, [])
    img = np.where(t <= synth.MAX_RANGE, t, 0.0).astype(np.float32)
    return img, phi


@pytest.mark.parametrize("H, W, top, bottom", [(64, 2048, 2.0, -24.8), (32, 1800, 10.0, -30.0),
                                               (128, 512, 2.0, -24.8)])
def test_flat_ground_fully_removed(H, W, top, bottom):
    img, phi = _flat_ground(H, W, top, bottom)
    mask, out = oracle.ground(img, synth.ground_tables(phi))
    valid = img > 0
    assert valid.sum() > 0
    assert (mask[valid] == 1).all()
    assert (mask[~valid] == 0).all()
    assert (out == 0).all()


def test_vertical_surfaces_kept():
    """Cylinders taller than the sensor show only vertical faces: none of their
    cells is ground, and the only ground cells kept are those directly above
    or below an object cell (a pair spanning two surfaces)."""
    phi = synth.elevations(64, 2.0, -24.8)
    rng = np.random.default_rng(9)
    objs = []
    for i in range(40):
        d = rng.uniform(4.0, 50.0)
        b = rng.uniform(0.0, 2 * math.pi)
        r = rng.uniform(0.3, 1.5)
        objs.append(synth._Obj(1, d * math.cos(b), d * math.sin(b), r, 0.0, 4.0, 0.0, r))
    t, sid = synth.raycast(phi, 1024, objs)
    img = np.where(t <= synth.MAX_RANGE, t, 0.0).astype(np.float32)
    mask, out = oracle.ground(img, synth.ground_tables(phi))
    obj = (sid > 0) & (img > 0)
    gnd = (sid == 0) & (img > 0)
    assert obj.sum() > 1000
    assert (mask[obj] == 0).all()
    np.testing.assert_array_equal(out[obj], img[obj])
    adj = np.zeros_like(gnd)
    adj[1:] |= obj[:-1]
    adj[:-1] |= obj[1:]
    kept = gnd & (mask == 0)
    assert not (kept & ~adj).any()


def _tilted_pair(d1, delta0, delta1, slope):
    """Range along the lower beam (elevation delta1) of the point B where the
    line through A = d1 (cos delta0, sin delta0) with the given slope angle
    (rising away from the sensor) meets that beam."""
    ax, az = d1 * math.cos(delta0), d1 * math.sin(delta0)
    ux, uz = math.cos(delta1), math.sin(delta1)
    # A + s (cos slope, sin slope) = t (ux, uz)
    cs, sn = math.cos(slope), math.sin(slope)
    det = cs * (-uz) - sn * (-ux)
    t = (cs * (-az) - sn * (-ax)) / det
    return t


@pytest.mark.parametrize("slope_deg, ground", [(0.0, True), (5.0, True), (-5.0, True), (9.0, True),
                                               (-9.0, True), (11.0, False), (-11.0, False),
                                               (30.0, False), (-30.0, False), (80.0, False)])
def test_tilted_plane_window(slope_deg, ground):
    """Eq. (2) with the +-10 degree window: a surface within 10 degrees of
    horizontal is ground, a steeper one is not (rows 15 degrees and more below
    the horizon, so the window is not clamped; the height line is lifted out
    of the way)."""
    H, W = 2, 3
    phi = np.deg2rad(np.array([-15.0, -15.4]))
    g = synth.ground_tables(phi)
    g.sensor_height = 0.0                       # z = d sin(delta) < 0 <= line
    d1 = 8.0
    d2 = _tilted_pair(d1, phi[0], phi[1], math.radians(slope_deg))
    assert d2 > 0
    img = np.array([[d1] * W, [d2] * W], dtype=np.float32)
    mask, _ = oracle.ground(img, g)
    assert (mask == (1 if ground else 0)).all()          # row 0 takes row 1's test


def test_obtuse_surface_angle_never_ground():
    """A lower cell farther out than the upper one along a steep pair gives a
    negative denominator (beta > 90 degrees): never horizontal."""
    phi = np.deg2rad(np.array([1.0, 0.6]))          # near the horizon: window reaches 0
    g = synth.ground_tables(phi)
    g.sensor_height = -100.0                        # height line out of the way
    img = np.array([[5.0, 5.0, 5.0], [9.0, 9.0, 9.0]], dtype=np.float32)
    mask, _ = oracle.ground(img, g)
    assert (mask == 0).all()


def test_first_row_and_missing_above_take_the_pair_below():
    img, phi = _flat_ground(16, 64, -10.0, -25.0)
    g = synth.ground_tables(phi)
    assert (img > 0).all()
    # row 0 has no row above: removed because rows 0-1 are a flat pair
    mask, _ = oracle.ground(img, g)
    assert (mask == 1).all()
    # a dropout above a cell: the cell takes its pair with the cell below
    hole = img.copy()
    hole[5, 10] = 0.0
    mask, out = oracle.ground(hole, g)
    assert mask[6, 10] == 1 and out[5, 10] == 0
    # ... unless that is missing too: an isolated cell spans no surface
    iso = img.copy()
    iso[4, 20] = 0.0
    iso[6, 20] = 0.0
    mask, out = oracle.ground(iso, g)
    assert mask[5, 20] == 0 and out[5, 20] == img[5, 20]
    # row 0 with row 1 missing is kept
    top = img.copy()
    top[1, 30] = 0.0
    mask, _ = oracle.ground(top, g)
    assert mask[0, 30] == 0 and mask[2, 30] == 1


@pytest.mark.parametrize("z0", [0.5, 1.0, 1.5])
def test_height_line(z0):
    """A horizontal plane z0 above the wheel plane is removed only beyond the
    distance where the 10-degree line from the wheel position passes z0."""
    H, W = 48, 8
    phi = np.deg2rad(np.linspace(-0.5, -45.0, H))
    g = synth.ground_tables(phi)
    hz = g.sensor_height - z0                        # plane z0 above the wheel plane, below the sensor
    d = (hz / np.sin(-phi)).astype(np.float32)       # every beam meets the plane
    img = np.repeat(d[:, None], W, axis=1)
    mask, _ = oracle.ground(img, g)
    x = d.astype(np.float64) * np.cos(phi)
    x_line = z0 / math.tan(math.radians(10.0))
    far = x > x_line * 1.01
    near = x < x_line * 0.99
    assert far.any() and near.any()
    assert (mask[far] == 1).all()
    assert (mask[near] == 0).all()


def test_non_measurements_copied_and_never_ground():
    img, phi = _flat_ground(8, 16, -10.0, -25.0)
    specials = np.array([0.0, -0.0, -1.0, np.nan, np.inf, -np.inf], dtype=np.float32)
    img[3, :6] = specials
    mask, out = oracle.ground(img, synth.ground_tables(phi))
    assert (mask[3, :6] == 0).all()
    np.testing.assert_array_equal(out[3, :6].view(np.uint32), specials.view(np.uint32))


def test_single_row_has_no_ground():
    img, phi = _flat_ground(1, 32, -10.0, -10.0)
    mask, out = oracle.ground(img, synth.ground_tables(phi))
    assert (mask == 0).all()
    np.testing.assert_array_equal(out, img)


@pytest.mark.parametrize("slope_deg, ground", [(9.5, True), (-9.5, True), (10.5, False), (-10.5, False)])
def test_tilted_plane_window_wide_pair(slope_deg, ground):
    """The same near the window's edges, with rows 4 degrees apart (so d1 and
    d2 differ by a quarter and every term of Eq. (2) matters)."""
    phi = np.deg2rad(np.array([-15.0, -19.0]))
    g = synth.ground_tables(phi)
    g.sensor_height = 0.0
    d1 = 8.0
    d2 = _tilted_pair(d1, phi[0], phi[1], math.radians(slope_deg))
    img = np.array([[d1] * 3, [d2] * 3], dtype=np.float32)
    mask, _ = oracle.ground(img, g)
    assert (mask == (1 if ground else 0)).all()


def test_flat_ground_uneven_row_spacing():
    """Row spacings alternating between 0.2 degrees and 12 to 22 degrees: each
    pair is tested against its own window (a neighbouring pair's window is
    more than 10 degrees off)."""
    phi = np.deg2rad(np.array([-3.0, -15.0, -15.2, -30.0, -30.2, -48.0, -48.2, -70.0, -70.2]))
    t, _ = synth.raycast(phi, 64, [])
    img = np.where(t <= synth.MAX_RANGE, t, 0.0).astype(np.float32)
    mask, _ = oracle.ground(img, synth.ground_tables(phi))
    valid = img > 0
    assert valid.all()
    assert (mask == 1).all()


@pytest.mark.parametrize("slope_deg", [15.0, -15.0])
def test_steep_pair_below_a_wide_gap(slope_deg):
    """Rows 1-2 span a 15-degree slope under a row 15 degrees higher: the pair
    is not ground (its own window is 18 -+ 10 degrees), whatever the window of
    the pair above (3 -+ 10 degrees, clamped at 0) would say."""
    phi = np.deg2rad(np.array([-3.0, -18.0, -18.4]))
    g = synth.ground_tables(phi)
    g.sensor_height = 0.0
    d1 = 6.0
    d2 = _tilted_pair(d1, phi[1], phi[2], math.radians(slope_deg))
    img = np.array([[30.0] * 3, [d1] * 3, [d2] * 3], dtype=np.float32)
    mask, _ = oracle.ground(img, g)
    assert (mask[2] == 0).all()
