"""Launch-shape autotuner.

For each shape class (H, W, skip depth) it times the three tile shapes the
kernels support (64, 128 or 256 columns per 8192-pixel tile) on a batch of
workload scenes of that shape (raycast objects and dropouts, as the mixed
batch draws them), by the throughput the serving and batch paths see:
batched launches of the batch overlapped on several streams, microseconds per
scan over the whole run.  It keeps the fastest.  It also times a plan of the
mixed-shape batch at several branch splits (flic_ctx_set_plan_parts: the
launch sequences per shape group, which decide how the groups' border passes
overlap) and keeps the fastest.  Last, since scans of different shapes share
launches (a mixed batch, the serving loop), it refines the per-shape tile
widths one shape at a time by the relaunch time of one plan over 256
mixed-shape scans, keeping a change only when it is at least 3 % faster.  The choices go to a
JSON cache keyed by GPU architecture; applying the cache installs them on a
context (per-shape tile rules, plan parts).  Labels never depend on either
choice, only speed does.

    python -m paper_2003_00575_amd.autotune --out flic_tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

CANDIDATES: Tuple[int, ...] = (64, 128, 256)
PLAN_PARTS: Tuple[int, ...] = (1, 2, 4)
PLAN_KEY = "_plan_parts"              # arch-level entry (not a shape)
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


def record_plan_parts(cache: Dict[str, Dict[str, dict]], arch: str, timings: Dict[int, float]) -> int:
    """Fastest plan split; ties go to fewer parts (fewer launches)."""
    if not timings:
        raise ValueError("no timings")
    choice = min(timings, key=lambda p: (timings[p], p))
    cache.setdefault(arch, {})[PLAN_KEY] = {
        "parts": choice, "us_per_plan": {str(k): round(v, 3) for k, v in sorted(timings.items())}}
    return choice


def rules_for(cache: Dict[str, Dict[str, dict]], arch: str) -> List[Tuple[int, int, int, int]]:
    return [(*parse_key(k), int(v["tile_w"])) for k, v in sorted(cache.get(arch, {}).items())
            if not k.startswith("_")]


def plan_parts_for(cache: Dict[str, Dict[str, dict]], arch: str) -> Optional[int]:
    entry = cache.get(arch, {}).get(PLAN_KEY)
    return None if entry is None else int(entry["parts"])


def apply(ctx, cache: Dict[str, Dict[str, dict]], arch: str) -> int:
    """Install the cached choices on a flic Context; returns how many tile
    rules (the plan split, when cached, is installed too)."""
    rules = rules_for(cache, arch)
    for H, W, N, tw in rules:
        ctx.set_tile_rule(H, W, N, tw)
    parts = plan_parts_for(cache, arch)
    if parts is not None:
        ctx.set_plan_parts(parts)
    return len(rules)


DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")


def apply_default(ctx, path: Optional[str] = None) -> int:
    """Install the shipped tile table (or the one at `path`) for this GPU, if
    it has an entry."""
    return apply(ctx, load_cache(path or DEFAULT_CACHE), gpu_arch())


def gpu_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def workload_scan(H: int, W: int, N: int, i: int, threshold: float = 0.5):
    """Scan i of a tuning batch: a raycast scene of this shape drawn as the
    mixed batch draws its scans (field of view of the matching mixed shape,
    else the 64-beam one; 40 objects and 10 % i.i.d. dropouts up to 64 rows,
    120 objects and 20 % bursts above)."""
    from . import synth
    top, bot = 2.0, -24.8
    for h, w, t, b in synth.MIXED_SHAPES:
        if (h, w) == (H, W):
            top, bot = t, b
    if H <= 64:
        return synth.synth_scan(H, W, top, bot, 40, "iid10", 9000 + i, threshold, N)
    return synth.synth_scan(H, W, top, bot, 120, "burst20", 9000 + i, threshold, N)


def _overlapped_us(launch, streams, reps: int) -> float:
    """Microseconds of `reps` rounds of launch(k, stream) on every stream,
    from one event before to one after all of them (stream 0 joins the rest)."""
    import torch
    s0 = streams[0]
    for k, st in enumerate(streams):                 # warm-up
        launch(k, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s0)
    for st in streams[1:]:
        st.wait_event(e0)
    for _ in range(reps):
        for k, st in enumerate(streams):
            launch(k, st)
    for st in streams[1:]:
        ev = torch.cuda.Event()
        ev.record(st)
        s0.wait_event(ev)
    e1.record(s0)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3


def time_shape(ctx, shape: Shape, n_scans: int = 32, reps: int = 8,
               candidates: Sequence[int] = CANDIDATES, n_streams: int = 3) -> Dict[int, float]:
    """Microseconds per scan, per candidate tile width, of batched launches of
    n_scans workload scenes overlapped on n_streams streams (each stream its
    own copy of the batch)."""
    import torch
    from . import flic
    H, W, N = shape
    host = [workload_scan(H, W, N, i) for i in range(n_scans)]
    arrs = [flic.Context.scan_array([flic.to_device(s) for s in host]) for _ in range(n_streams)]
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    out: Dict[int, float] = {}
    previous = ctx.tile_for(H, W, N)
    try:
        for tw in candidates:
            ctx.set_tile_rule(H, W, N, tw)
            us = _overlapped_us(lambda k, st: ctx.cluster_batched_array(arrs[k], st), streams, reps)
            out[tw] = us / (reps * n_streams * n_scans)
    finally:
        ctx.set_tile_rule(H, W, N, 0)
        if previous != ctx.tile_for(H, W, N):
            ctx.set_tile_rule(H, W, N, previous)
    return out


class MixedPlanTimer:
    """Relaunch time of one plan over n_scans mixed-shape scans (the current
    rules of the context) on one stream: the median over `repeats` timings of
    `reps` back-to-back relaunches (single timings vary by a few per cent)."""

    def __init__(self, ctx, n_scans: int = 256, reps: int = 20, repeats: int = 5):
        import torch
        from . import flic, synth
        self.ctx, self.reps, self.repeats = ctx, reps, repeats
        host = [synth.mixed_scan(i) for i in range(n_scans)]
        self.shapes = sorted({(s.H, s.W, s.skip_depth) for s in host})
        self.devs = [flic.to_device(s) for s in host]
        self.stream = torch.cuda.Stream()

    def us_per_plan(self) -> float:
        plan = self.ctx.plan(self.devs)
        try:
            times = sorted(_overlapped_us(lambda k, st: plan.relaunch(st), [self.stream], self.reps) / self.reps
                           for _ in range(self.repeats))
        finally:
            plan.close()
        return times[len(times) // 2]


def time_plan_parts(ctx, n_scans: int = 256, candidates: Sequence[int] = PLAN_PARTS,
                    timer: Optional[MixedPlanTimer] = None) -> Dict[int, float]:
    """Microseconds per relaunch of the mixed-shape plan, per plan split."""
    timer = timer or MixedPlanTimer(ctx, n_scans)
    out: Dict[int, float] = {}
    for parts in candidates:
        ctx.set_plan_parts(parts)
        out[parts] = timer.us_per_plan()
    ctx.set_plan_parts(1)
    return out


def refine_in_mix(ctx, cache: Dict[str, Dict[str, dict]], arch: str, timer: MixedPlanTimer,
                  candidates: Sequence[int] = CANDIDATES, min_gain: float = 0.03) -> float:
    """Coordinate descent over the tile widths of the mixed plan's shapes:
    one shape at a time, each other width is tried and kept when the plan
    relaunches at least min_gain faster.  Updates the cache; returns the
    final microseconds per plan."""
    apply(ctx, cache, arch)
    best = timer.us_per_plan()
    for H, W, N in timer.shapes:
        key = shape_key(H, W, N)
        if key not in cache.get(arch, {}):
            continue
        entry = cache[arch][key]
        plan_us = {str(entry["tile_w"]): round(best, 3)}
        for tw in candidates:
            if tw == entry["tile_w"]:
                continue
            ctx.set_tile_rule(H, W, N, tw)
            us = timer.us_per_plan()
            plan_us[str(tw)] = round(us, 3)
            if us < best * (1.0 - min_gain):
                best = us
                entry["tile_w"] = tw
        ctx.set_tile_rule(H, W, N, entry["tile_w"])
        entry["us_per_mixed_plan"] = dict(sorted(plan_us.items()))
    return best


def tune(ctx, shapes: Iterable[Shape], cache_path: Optional[str] = None,
         n_scans: int = 32, reps: int = 8, plan_scans: int = 256) -> Dict[str, Dict[str, dict]]:
    arch = gpu_arch()
    cache = load_cache(cache_path) if cache_path else {}
    for shape in shapes:
        record(cache, arch, shape, time_shape(ctx, shape, n_scans, reps))
    apply(ctx, cache, arch)                          # plans time with the tile choices
    if plan_scans > 0:
        timer = MixedPlanTimer(ctx, plan_scans)
        refine_in_mix(ctx, cache, arch, timer)
        record_plan_parts(cache, arch, time_plan_parts(ctx, timer=timer))
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
    ap.add_argument("--plan-scans", type=int, default=256,
                    help="mixed-shape scans in the plan-split timing (0: skip it)")
    args = ap.parse_args()
    shapes = [(H, W, args.skip) for H, W, _, _ in synth.MIXED_SHAPES]
    ctx = flic.Context(0)
    cache = tune(ctx, shapes, args.out, n_scans=args.scans, plan_scans=args.plan_scans)
    print(json.dumps(cache, indent=1, sort_keys=True))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
