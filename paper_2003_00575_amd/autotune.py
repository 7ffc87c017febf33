"""Tile-shape autotuner.

For each shape class (H, W, skip depth) it times the three tile shapes the
kernels support (64, 128 or 256 columns per 8192-pixel tile) on a batch of
synthetic scans of that shape, keeps the fastest, and records the choice in a
JSON cache keyed by GPU architecture.  Applying the cache installs the
choices as per-shape tile rules on a context (flic_ctx_set_tile_rule); labels
never depend on the tile shape, only speed does.

    python -m paper_2003_00575_amd.autotune --out flic_tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

CANDIDATES: Tuple[int, ...] = (64, 128, 256)
Shape = Tuple[int, int, int]          # (H, W, skip depth)


def shape_key(H: int, W: int, N: int) -> str:
    return f"{H}x{W}xN{N}"


def parse_key(key: str) -> Shape:
    hw, n = key.split("xN")
    h, w = hw.split("x")
    return int(h), int(w), int(n)


def best_choice(timings: Dict[int, float]) -> int:
    """Fastest candidate; ties go to the wider tile (fewer borders)."""
    if not timings:
        raise ValueError("no timings")
    return min(timings, key=lambda t: (timings[t], -t))


def load_cache(path: str) -> Dict[str, Dict[str, dict]]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not a tile cache")
    return data


def save_cache(path: str, cache: Dict[str, Dict[str, dict]]) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def record(cache: Dict[str, Dict[str, dict]], arch: str, shape: Shape,
           timings: Dict[int, float]) -> int:
    choice = best_choice(timings)
    cache.setdefault(arch, {})[shape_key(*shape)] = {
        "tile_w": choice, "us_per_scan": {str(k): round(v, 3) for k, v in sorted(timings.items())}}
    return choice


def rules_for(cache: Dict[str, Dict[str, dict]], arch: str) -> List[Tuple[int, int, int, int]]:
    return [(*parse_key(k), int(v["tile_w"])) for k, v in sorted(cache.get(arch, {}).items())]


def apply(ctx, cache: Dict[str, Dict[str, dict]], arch: str) -> int:
    """Install the cached choices on a flic Context; returns how many."""
    rules = rules_for(cache, arch)
    for H, W, N, tw in rules:
        ctx.set_tile_rule(H, W, N, tw)
    return len(rules)


DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")


def apply_default(ctx) -> int:
    """Install the shipped tile table for this GPU (if it has an entry)."""
    return apply(ctx, load_cache(DEFAULT_CACHE), gpu_arch())


def gpu_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def time_shape(ctx, shape: Shape, n_scans: int = 32, reps: int = 8,
               candidates: Sequence[int] = CANDIDATES) -> Dict[int, float]:
    """Mean microseconds per scan of the three passes, per candidate tile width
    (batched launches, HIP events around each pass)."""
    import torch
    from . import flic, synth
    H, W, N = shape
    scans = []
    for i in range(n_scans):
        s = synth.random_scan(H, W, N, seed=9000 + i, threshold=0.5, p_invalid=0.15)
        scans.append(flic.to_device(s))
    arr = flic.Context.scan_array(scans)
    out: Dict[int, float] = {}
    previous = ctx.tile_for(H, W, N)
    try:
        for tw in candidates:
            ctx.set_tile_rule(H, W, N, tw)
            ctx.cluster_batched_array(arr)            # warm-up (allocates scratch)
            torch.cuda.synchronize()
            ctx.set_pass_timing(True)
            ctx.pass_times()
            for _ in range(reps):
                ctx.cluster_batched_array(arr)
            ms, n = ctx.pass_times()
            ctx.set_pass_timing(False)
            out[tw] = sum(ms) / max(1, n) * 1e3 / n_scans
    finally:
        ctx.set_tile_rule(H, W, N, 0)
        if previous != ctx.tile_for(H, W, N):
            ctx.set_tile_rule(H, W, N, previous)
    return out


def tune(ctx, shapes: Iterable[Shape], cache_path: Optional[str] = None,
         n_scans: int = 32, reps: int = 8) -> Dict[str, Dict[str, dict]]:
    arch = gpu_arch()
    cache = load_cache(cache_path) if cache_path else {}
    for shape in shapes:
        record(cache, arch, shape, time_shape(ctx, shape, n_scans, reps))
    if cache_path:
        save_cache(cache_path, cache)
    apply(ctx, cache, arch)
    return cache


def main() -> int:
    from . import flic, synth
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default="flic_tiles.json")
    ap.add_argument("--skip", type=int, default=3)
    ap.add_argument("--scans", type=int, default=32)
    args = ap.parse_args()
    shapes = [(H, W, args.skip) for H, W, _, _ in synth.MIXED_SHAPES]
    ctx = flic.Context(0)
    cache = tune(ctx, shapes, args.out, n_scans=args.scans)
    print(json.dumps(cache, indent=1, sort_keys=True))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
