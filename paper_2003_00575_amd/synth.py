"""Seeded synthetic Lidar range images and angle tables.

This module only builds inputs: it raycasts a simple scene (ground plane plus
boxes and vertical cylinders) from a sensor at the origin straight into an
H x W range image, applies noise and dropouts, and tabulates cos(alpha) for
every neighbour offset.  It contains none of the clustering arithmetic; both
the GPU path and the CPU oracle consume what it produces.

Geometry follows the paper's sensor model (Section III): row r is a laser
channel at elevation phi_r, column c is the azimuth 2*pi*c/W, a range of 0
marks a missing measurement.  The per-row / per-column angles between
neighbouring measurements are caller data that a sensor manufacturer would
supply (Section III.B, Eq. 4); here they come from the synthetic elevations.

Randomness: one numpy PCG64 generator per scan, seeded by the caller.  Draw
order is fixed (objects, then noise, then dropouts), so a seed fully
determines the bytes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

GROUND_Z = -1.73          # metres below the sensor
MAX_RANGE = 120.0         # metres; no hit or farther -> 0 (missing)
MIN_RANGE = 0.5
NOISE_SIGMA = 0.02

# (H, W, top elevation deg, bottom elevation deg) of the mixed-shape set.
MIXED_SHAPES: Tuple[Tuple[int, int, float, float], ...] = (
    (16, 1024, 15.0, -15.0),
    (32, 1800, 10.0, -30.0),
    (64, 2048, 2.0, -24.8),
    (128, 2048, 2.0, -24.8),
    (128, 4096, 2.0, -24.8),
)


@dataclasses.dataclass
class Scan:
    """One range image with its angle tables and clustering parameters.

    range_img: float32 [H, W], metres, 0 = missing.
    cos_v:     float32 [N, H]; cos_v[k-1, r] = cos(angle between rows r and r+k),
               entries with r >= H-k are unused and hold NaN.
    cos_h:     float32 [N, W]; cos_h[k-1, c] = cos(angle between columns c and
               (c+k) mod W).
    threshold: metres.   skip_depth: N >= 1.
    object_id: int32 [H, W] ground-truth surface id (-1 none, 0 ground,
               i+1 object i) before dropouts; used only for quality metrics.
    """
    range_img: np.ndarray
    cos_v: np.ndarray
    cos_h: np.ndarray
    threshold: float
    skip_depth: int
    object_id: Optional[np.ndarray] = None
    seed: Optional[int] = None
    phi: Optional[np.ndarray] = None      # row elevations (radians, float64), when known

    @property
    def H(self) -> int:
        return int(self.range_img.shape[0])

    @property
    def W(self) -> int:
        return int(self.range_img.shape[1])


# ---------------------------------------------------------------------------
# Angles and tables
# ---------------------------------------------------------------------------

def elevations(H: int, top_deg: float, bottom_deg: float,
               jitter_deg: float = 0.0,
               rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """Row elevations in radians (float64), row 0 = top, uniform spacing,
    optionally perturbed per row by U(-jitter, +jitter) degrees."""
    if H == 1:
        phi = np.array([top_deg], dtype=np.float64)
    else:
        phi = top_deg - np.arange(H, dtype=np.float64) * (top_deg - bottom_deg) / (H - 1)
    if jitter_deg > 0.0:
        assert rng is not None
        phi = phi + rng.uniform(-jitter_deg, jitter_deg, size=H)
    return np.deg2rad(phi)


def make_tables(phi: np.ndarray, W: int, N: int) -> Tuple[np.ndarray, np.ndarray]:
    """cos tables as float32, computed in double then rounded once.

    cos_v[k-1, r] = cos(phi_r - phi_{r+k}) for r + k < H, NaN otherwise.
    cos_h[k-1, c] = cos(2*pi*k/W) (uniform azimuth spacing).
    """
    H = phi.shape[0]
    cos_v = np.full((N, H), np.nan, dtype=np.float32)
    for k in range(1, N + 1):
        if k < H:
            cos_v[k - 1, : H - k] = np.cos(phi[: H - k] - phi[k:]).astype(np.float32)
    cos_h = np.empty((N, W), dtype=np.float32)
    for k in range(1, N + 1):
        cos_h[k - 1, :] = np.float32(math.cos(2.0 * math.pi * k / W))
    return cos_v, cos_h


# ---------------------------------------------------------------------------
# Scene + raycasting
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class _Obj:
    kind: int          # 0 box, 1 cylinder
    cx: float
    cy: float
    a: float           # box length / cylinder radius
    b: float           # box width (unused for cylinders)
    h: float           # height
    yaw: float         # box yaw
    r_bound: float     # horizontal bounding-circle radius


def _draw_objects(n: int, rng: np.random.Generator) -> List[_Obj]:
    objs: List[_Obj] = []
    while len(objs) < n:
        if rng.uniform() < 0.5:
            L, Wd, Ht = rng.uniform(0.5, 5.0, size=3)
            yaw = rng.uniform(0.0, math.pi)
            kind, a, b, rb = 0, float(L), float(Wd), 0.5 * math.hypot(L, Wd)
        else:
            dia, Ht = rng.uniform(0.5, 5.0, size=2)
            yaw = 0.0
            kind, a, b, rb = 1, 0.5 * float(dia), 0.0, 0.5 * float(dia)
        dist = rng.uniform(3.0, 60.0)
        bearing = rng.uniform(0.0, 2.0 * math.pi)
        if dist - rb < 0.5:          # footprint too close to the sensor: redraw
            continue
        objs.append(_Obj(kind, dist * math.cos(bearing), dist * math.sin(bearing),
                         a, b, float(Ht), float(yaw), rb))
    return objs


def _cols_covering(o: _Obj, W: int) -> np.ndarray:
    """Columns whose azimuth can intersect the object's bounding circle."""
    d = math.hypot(o.cx, o.cy)
    half = math.asin(min(1.0, o.r_bound / d)) + 2.0 * math.pi / W
    bearing = math.atan2(o.cy, o.cx)
    lo = math.floor((bearing - half) * W / (2.0 * math.pi))
    hi = math.ceil((bearing + half) * W / (2.0 * math.pi))
    return np.arange(lo, hi + 1) % W


def _hit_box(o: _Obj, dx, dy, dz):
    cs, sn = math.cos(o.yaw), math.sin(o.yaw)
    lx = dx * cs + dy * sn
    ly = -dx * sn + dy * cs
    ox = -(o.cx * cs + o.cy * sn)
    oy = -(-o.cx * sn + o.cy * cs)
    oz = 0.0
    lo = (-0.5 * o.a, -0.5 * o.b, GROUND_Z)
    hi = (0.5 * o.a, 0.5 * o.b, GROUND_Z + o.h)
    tmin = np.full(dx.shape, -np.inf)
    tmax = np.full(dx.shape, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        for d, orig, l, h in ((lx, ox, lo[0], hi[0]), (ly, oy, lo[1], hi[1]),
                              (dz, oz, lo[2], hi[2])):
            inv = 1.0 / d
            t1 = (l - orig) * inv
            t2 = (h - orig) * inv
            near = np.minimum(t1, t2)
            far = np.maximum(t1, t2)
            par = d == 0.0
            inside = (orig >= l) & (orig <= h)
            near = np.where(par, np.where(inside, -np.inf, np.inf), near)
            far = np.where(par, np.where(inside, np.inf, -np.inf), far)
            tmin = np.maximum(tmin, near)
            tmax = np.minimum(tmax, far)
    hit = (tmax >= tmin) & (tmin > 0.0)
    return np.where(hit, tmin, np.inf)


def _hit_cylinder(o: _Obj, dx, dy, dz):
    R = o.a
    zb, zt = GROUND_Z, GROUND_Z + o.h
    ox, oy = -o.cx, -o.cy
    a = dx * dx + dy * dy
    b = 2.0 * (ox * dx + oy * dy)
    c = ox * ox + oy * oy - R * R
    disc = b * b - 4.0 * a * c
    t = np.full(dx.shape, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        sq = np.sqrt(np.maximum(disc, 0.0))
        t_side = (-b - sq) / (2.0 * a)
        z = t_side * dz
        ok = (disc >= 0.0) & (a > 0.0) & (t_side > 0.0) & (z >= zb) & (z <= zt)
        t = np.where(ok, t_side, t)
        for zc in (zt, zb):
            tc = zc / dz
            px = tc * dx + ox
            py = tc * dy + oy
            okc = (dz != 0.0) & (tc > 0.0) & (px * px + py * py <= R * R)
            t = np.where(okc & (tc < t), tc, t)
    return t


def raycast(phi: np.ndarray, W: int, objs: Sequence[_Obj]) -> Tuple[np.ndarray, np.ndarray]:
    """Nearest positive hit distance (float64, inf = none) and surface id."""
    H = phi.shape[0]
    theta = 2.0 * math.pi * np.arange(W) / W
    cphi, sphi = np.cos(phi), np.sin(phi)
    dz_row = sphi
    with np.errstate(divide="ignore"):
        tg = np.where(dz_row < 0.0, GROUND_Z / dz_row, np.inf)
    t_best = np.repeat(tg[:, None], W, axis=1)
    sid = np.where(np.isfinite(t_best), 0, -1).astype(np.int32)
    cth, sth = np.cos(theta), np.sin(theta)
    for i, o in enumerate(objs):
        cols = _cols_covering(o, W)
        dx = cphi[:, None] * cth[None, cols]
        dy = cphi[:, None] * sth[None, cols]
        dz = np.broadcast_to(sphi[:, None], dx.shape)
        t = _hit_box(o, dx, dy, dz) if o.kind == 0 else _hit_cylinder(o, dx, dy, dz)
        cur = t_best[:, cols]
        better = t < cur
        if better.any():
            t_best[:, cols] = np.where(better, t, cur)
            s = sid[:, cols]
            sid[:, cols] = np.where(better, i + 1, s)
    return t_best, sid


def _finish_ranges(t: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    hit = t <= MAX_RANGE
    noise = rng.normal(0.0, NOISE_SIGMA, size=t.shape)
    r = np.where(hit, np.clip(t + noise, MIN_RANGE, MAX_RANGE), 0.0)
    return r.astype(np.float32)


def dropouts_iid(img: np.ndarray, p: float, rng: np.random.Generator) -> None:
    img[rng.uniform(size=img.shape) < p] = 0.0


def dropouts_bursts(img: np.ndarray, frac: float, rng: np.random.Generator) -> None:
    """Zero axis-aligned rectangles of U{1..4} rows x U{8..64} columns (wrapping
    horizontally, clipped vertically) until >= frac of the pixels are covered."""
    H, W = img.shape
    covered = np.zeros((H, W), dtype=bool)
    need = int(math.ceil(frac * H * W))
    n = 0
    while n < need:
        h = int(rng.integers(1, 5))
        w = int(rng.integers(8, 65))
        r0 = int(rng.integers(0, H))
        c0 = int(rng.integers(0, W))
        idx = np.ix_(np.arange(r0, min(H, r0 + h)), np.arange(c0, c0 + w) % W)
        blk = covered[idx]
        n += int(blk.size - blk.sum())
        covered[idx] = True
    img[covered] = 0.0


def synth_scan(H: int, W: int, top_deg: float, bottom_deg: float, n_objects: int,
               dropout: str, seed: int, threshold: float, skip_depth: int,
               jitter_deg: float = 0.0) -> Scan:
    """One raycast scene.  dropout is 'iid10' (Bernoulli 0.10) or 'burst20'
    (clustered rectangles until 20 % covered)."""
    rng = np.random.default_rng(seed)
    phi = elevations(H, top_deg, bottom_deg, jitter_deg, rng)
    objs = _draw_objects(n_objects, rng)
    t, sid = raycast(phi, W, objs)
    img = _finish_ranges(t, rng)
    if dropout == "iid10":
        dropouts_iid(img, 0.10, rng)
    elif dropout == "burst20":
        dropouts_bursts(img, 0.20, rng)
    elif dropout != "none":
        raise ValueError(dropout)
    cos_v, cos_h = make_tables(phi, W, skip_depth)
    return Scan(img, cos_v, cos_h, float(threshold), int(skip_depth), sid, seed, phi)


@dataclasses.dataclass
class GroundTables:
    """Per-row sensor tables for ground extraction, float32 [H] each:
    sin_a / cos_a of the angle between rows r-1 and r, the window
    [tan_lo, tan_hi] of tan(beta) for that pair to lie on a horizontal
    surface (entries 0 unused, NaN), sin_d / cos_d of row r's elevation; the
    sensor height over the wheel plane and the slope of the height line."""
    sin_a: np.ndarray
    cos_a: np.ndarray
    tan_lo: np.ndarray
    tan_hi: np.ndarray
    sin_d: np.ndarray
    cos_d: np.ndarray
    sensor_height: float
    tan_theta: float


def ground_tables(phi: np.ndarray, theta_deg: float = 10.0,
                  sensor_height: float = -GROUND_Z) -> GroundTables:
    """Tables for elevations phi (radians, row 0 = top), computed in double
    and rounded once to float32.  A horizontal surface meets the upper beam
    of a row pair at the beam's angle below the horizontal, -phi_{r-1}; the
    window is that angle -+ theta, its lower end clamped at 0 (a surface
    angle is never negative)."""
    H = phi.shape[0]
    th = math.radians(theta_deg)
    nan = np.full(H, np.nan)
    a = phi[:-1] - phi[1:]
    beam = -phi[:-1]
    sin_a, cos_a, lo, hi = nan.copy(), nan.copy(), nan.copy(), nan.copy()
    sin_a[1:], cos_a[1:] = np.sin(a), np.cos(a)
    lo[1:] = np.tan(np.maximum(beam - th, 0.0))
    hi[1:] = np.tan(beam + th)
    f = lambda x: np.asarray(x, dtype=np.float64).astype(np.float32)
    return GroundTables(f(sin_a), f(cos_a), f(lo), f(hi), f(np.sin(phi)), f(np.cos(phi)),
                        float(np.float32(sensor_height)), float(np.float32(math.tan(th))))


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def single_scan(seed: int = 1) -> Scan:
    """64 x 2048, FOV +2/-24.8 deg, 40 objects, 10 % i.i.d. dropouts, T=0.5 m, N=3."""
    return synth_scan(64, 2048, 2.0, -24.8, 40, "iid10", seed, 0.5, 3)


def large_batch_scan(i: int, threshold: float = 0.5) -> Scan:
    """Scan i of the 64 x (128 x 2048) batch: 120 objects, 20 % burst dropouts, N=3."""
    return synth_scan(128, 2048, 2.0, -24.8, 120, "burst20", 1000 + i, threshold, 3)


def mixed_scan(i: int) -> Scan:
    """Scan i of the 256-scan uneven batch: shape i mod 5, own tables
    (per-row elevation jitter +-0.05 deg), T ~ U{0.3,0.5,0.8,1.0}, N=3."""
    H, W, top, bot = MIXED_SHAPES[i % 5]
    seed = 2000 + i
    trng = np.random.default_rng(seed + 7_000_000)
    T = float(trng.choice([0.3, 0.5, 0.8, 1.0]))
    if H <= 64:
        return synth_scan(H, W, top, bot, 40, "iid10", seed, T, 3, jitter_deg=0.05)
    return synth_scan(H, W, top, bot, 120, "burst20", seed, T, 3, jitter_deg=0.05)


def sensor_frame(sensor: int, frame: int, threshold: float) -> Scan:
    """Frame f of simulated sensor s (shape s mod 5), N=3."""
    H, W, top, bot = MIXED_SHAPES[sensor % 5]
    seed = 3000 + 100000 * sensor + frame
    if H <= 64:
        return synth_scan(H, W, top, bot, 40, "iid10", seed, threshold, 3, jitter_deg=0.0)
    return synth_scan(H, W, top, bot, 120, "burst20", seed, threshold, 3, jitter_deg=0.0)


# ---------------------------------------------------------------------------
# Closed-form stress patterns (64 x 4096 by default)
# ---------------------------------------------------------------------------

def _flat(mask: np.ndarray, seed: int, base: float = 5.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    img = (base + rng.uniform(0.0, 0.01, size=mask.shape)).astype(np.float32)
    img[~mask] = 0.0
    return img


def pattern_serpentine_rows(H: int = 64, W: int = 4096, seed: int = 0) -> np.ndarray:
    """Lanes on rows 0, 6, 12, ..., valid on columns 0..W-6; the rows between
    lane i and lane i+1 are valid only at column W-6 (i even) or 0 (i odd).
    One component when N <= 5."""
    m = np.zeros((H, W), dtype=bool)
    lanes = list(range(0, H, 6))
    for i, r in enumerate(lanes):
        m[r, : W - 5] = True
        if i + 1 < len(lanes):
            col = W - 6 if i % 2 == 0 else 0
            m[r: lanes[i + 1] + 1, col] = True
    return _flat(m, seed)


def pattern_serpentine_cols(H: int = 64, W: int = 4096, seed: int = 0) -> np.ndarray:
    """Lanes on columns 0, 6, ..., valid on all rows; the columns between lane
    j and j+1 are valid only in row H-1 (j even) or row 0 (j odd); columns past
    the last lane stay empty (seam gap >= 6).  One component when N <= 5."""
    m = np.zeros((H, W), dtype=bool)
    lanes = list(range(0, W - 9, 6))
    for j, c in enumerate(lanes):
        m[:, c] = True
        if j + 1 < len(lanes):
            row = H - 1 if j % 2 == 0 else 0
            m[row, c: lanes[j + 1] + 1] = True
    return _flat(m, seed)


def pattern_checkerboard(H: int = 64, W: int = 4096, seed: int = 0) -> np.ndarray:
    """Valid iff (r + c) is even."""
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    return _flat(((r + c) % 2) == 0, seed)


def pattern_wrap_runs(H: int = 64, W: int = 4096, seed: int = 0) -> np.ndarray:
    """Row r holds one run over columns [W-a_r, W-1] U [0, b_r-1] at range
    5 + 1.5 r metres (rows never connect to each other for T <= 1.0)."""
    rng = np.random.default_rng(seed)
    img = np.zeros((H, W), dtype=np.float32)
    for r in range(H):
        a = int(rng.integers(1, 513))
        b = int(rng.integers(1, 513))
        v = np.float32(5.0 + 1.5 * r)
        img[r, W - a:] = v
        img[r, :b] = v
    return img


def pattern_all_valid(H: int = 64, W: int = 4096, seed: int = 0) -> np.ndarray:
    return _flat(np.ones((H, W), dtype=bool), seed)


STRESS_PATTERNS = {
    "serpentine_rows": pattern_serpentine_rows,
    "serpentine_cols": pattern_serpentine_cols,
    "checkerboard": pattern_checkerboard,
    "wrap_runs": pattern_wrap_runs,
    "all_valid": pattern_all_valid,
}


def stress_scan(name: str, threshold: float, skip_depth: int, seed: int = 0,
                H: int = 64, W: int = 4096) -> Scan:
    phi = elevations(H, 2.0, -24.8)
    img = STRESS_PATTERNS[name](H, W, seed)
    cos_v, cos_h = make_tables(phi, W, skip_depth)
    return Scan(img, cos_v, cos_h, float(threshold), int(skip_depth), None, seed)


def random_scan(H: int, W: int, N: int, seed: int, threshold: float = 0.5,
                p_invalid: float = 0.2, spread: float = 0.6,
                angle_jitter: float = 0.5) -> Scan:
    """Unstructured random image for parity tests: ranges 5 +- spread metres
    with i.i.d. invalid pixels (exact zeros).  Angles: rows 0.4 deg apart and
    columns 0.09 deg apart, each neighbour angle scaled per row / per column by
    1 + U(-angle_jitter, angle_jitter), so every table entry differs."""
    rng = np.random.default_rng(seed)
    img = (5.0 + rng.uniform(-spread, spread, size=(H, W))).astype(np.float32)
    img[rng.uniform(size=(H, W)) < p_invalid] = 0.0
    step_v = np.deg2rad(0.4) * (1.0 + rng.uniform(-angle_jitter, angle_jitter, size=H))
    step_h = np.deg2rad(0.09) * (1.0 + rng.uniform(-angle_jitter, angle_jitter, size=W))
    phi = -np.concatenate([[0.0], np.cumsum(step_v[:-1])])
    cos_v, _ = make_tables(phi, W, N)
    theta = np.concatenate([[0.0], np.cumsum(step_h)])      # W + 1 entries
    cos_h = np.empty((N, W), dtype=np.float32)
    for k in range(1, N + 1):
        c = np.arange(W)
        lo, hi = c, c + k
        span = np.where(hi <= W, theta[np.minimum(hi, W)] - theta[lo],
                        theta[W] - theta[lo] + theta[(hi - W) % (W + 1)])
        cos_h[k - 1] = np.cos(span).astype(np.float32)
    return Scan(img, cos_v, cos_h, float(threshold), int(N), None, seed)
