"""Independent checking tools for the tests (no clustering code of the oracle or
the GPU library is reused here): union-find, canonical partitions, explicit-point
brute force, and the golden fixture reader."""
from __future__ import annotations

import math
import os
from typing import Dict, List, Tuple

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U32 = 2.0 ** -24   # unit roundoff of binary32


class UnionFind:
    def __init__(self, n: int):
        self.p = list(range(n))

    def find(self, x: int) -> int:
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a: int, b: int) -> None:
        ra, rb = self.find(a), self.find(b)
        if ra != rb:
            self.p[max(ra, rb)] = min(ra, rb)


def canonical(labels: np.ndarray) -> np.ndarray:
    """Relabel any partition (-1 = unlabelled) so each class gets its minimum
    linear index."""
    flat = labels.reshape(-1)
    out = np.full(flat.shape, -1, dtype=np.int64)
    first: Dict[int, int] = {}
    for i, v in enumerate(flat.tolist()):
        if v < 0:
            continue
        if v not in first:
            first[v] = i
        out[i] = first[v]
    return out.reshape(labels.shape)


def canonical_fast(labels: np.ndarray) -> np.ndarray:
    flat = labels.reshape(-1).astype(np.int64)
    out = np.full(flat.shape, -1, dtype=np.int64)
    m = flat >= 0
    if m.any():
        vals = flat[m]
        idx = np.nonzero(m)[0]
        uniq, inv = np.unique(vals, return_inverse=True)
        mins = np.full(uniq.shape, np.iinfo(np.int64).max)
        np.minimum.at(mins, inv, idx)
        out[m] = mins[inv]
    return out.reshape(labels.shape)


def is_measurement(r: np.ndarray) -> np.ndarray:
    return (r > 0) & np.isfinite(r)


def neighbour_pairs(H: int, W: int, N: int) -> List[Tuple[int, int, str, int]]:
    """All unordered pixel pairs satisfying the neighbour predicate, found by
    scanning every pair (not by a stencil): same column and 1 <= dr <= N, or
    same row and the forward column distance (c2 - c1) mod W in 1..N."""
    out = []
    P = H * W
    for p in range(P):
        r1, c1 = divmod(p, W)
        for q in range(P):
            if q == p:
                continue
            r2, c2 = divmod(q, W)
            if c1 == c2 and 1 <= r2 - r1 <= N:
                out.append((p, q, "v", r2 - r1))
            elif r1 == r2 and 1 <= (c2 - c1) % W <= N:
                out.append((p, q, "h", (c2 - c1) % W))
    return out


def explicit_points_distance(d1: float, d2: float, cos_alpha: float) -> float:
    """Distance between A = (d1, 0, 0) and B = d2 * (cos a, sin a, 0), in
    float64 (the triangle O, A, B of the paper's Fig. 3b)."""
    a = math.acos(max(-1.0, min(1.0, float(cos_alpha))))
    ax, ay = float(d1), 0.0
    bx, by = float(d2) * math.cos(a), float(d2) * math.sin(a)
    return math.sqrt((ax - bx) ** 2 + (ay - by) ** 2)


def read_golden(name: str) -> Dict[str, object]:
    """Read a golden text fixture: `key: value` scalars and `key:` followed by
    whitespace-separated matrix rows up to a blank line; `#` starts a comment."""
    path = os.path.join(GOLDEN, name)
    data: Dict[str, object] = {}
    key = None
    rows: List[List[float]] = []
    with open(path) as f:
        for raw in f:
            line = raw.split("#", 1)[0].rstrip()
            if not line.strip():
                if key is not None:
                    data[key] = np.array(rows)
                    key, rows = None, []
                continue
            if key is None and ":" in line:
                k, v = line.split(":", 1)
                k, v = k.strip(), v.strip()
                if v:
                    data[k] = v
                else:
                    key, rows = k, []
                continue
            rows.append([float(x) for x in line.split()])
    if key is not None:
        data[key] = np.array(rows)
    return data
