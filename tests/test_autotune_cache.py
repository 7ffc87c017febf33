"""Autotuner bookkeeping on the CPU: choice rule, cache format, round trip."""
from paper_2003_00575_amd import autotune


def test_best_choice_prefers_fastest_then_wider():
    assert autotune.best_choice({64: 3.0, 128: 2.0, 256: 2.5}) == 128
    assert autotune.best_choice({64: 2.0, 128: 2.0, 256: 2.0}) == 256


def test_cache_round_trip(tmp_path):
    cache = {}
    autotune.record(cache, "gfx950", (128, 2048, 3), {64: 1.0, 128: 1.5, 256: 2.0})
    autotune.record(cache, "gfx950", (16, 1024, 3), {64: 3.0, 128: 2.0, 256: 1.0})
    autotune.record(cache, "gfx942", (16, 1024, 3), {64: 1.0, 128: 2.0, 256: 3.0})
    p = str(tmp_path / "t.json")
    autotune.save_cache(p, cache)
    back = autotune.load_cache(p)
    assert back == cache
    assert autotune.rules_for(back, "gfx950") == [(128, 2048, 3, 64), (16, 1024, 3, 256)]
    assert autotune.rules_for(back, "gfx942") == [(16, 1024, 3, 64)]
    assert autotune.parse_key(autotune.shape_key(32, 1800, 5)) == (32, 1800, 5)
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


class _FakeCtx:
    def __init__(self):
        self.rules, self.parts = [], None

    def set_tile_rule(self, H, W, N, tw):
        self.rules.append((H, W, N, tw))

    def set_plan_parts(self, parts):
        self.parts = parts


def test_plan_parts_entry(tmp_path):
    cache = {}
    autotune.record(cache, "gfx950", (128, 2048, 3), {64: 1.0, 128: 1.5, 256: 2.0})
    # fastest split wins; a tie goes to fewer parts
    assert autotune.record_plan_parts(cache, "gfx950", {1: 300.0, 2: 280.0, 4: 310.0}) == 2
    assert autotune.record_plan_parts(cache, "gfx950", {1: 300.0, 2: 300.0, 4: 310.0}) == 1
    p = str(tmp_path / "t.json")
    autotune.save_cache(p, cache)
    back = autotune.load_cache(p)
    # the arch-level entry is not a shape rule
    assert autotune.rules_for(back, "gfx950") == [(128, 2048, 3, 64)]
    assert autotune.plan_parts_for(back, "gfx950") == 1
    assert autotune.plan_parts_for(back, "gfx942") is None
    ctx = _FakeCtx()
    assert autotune.apply(ctx, back, "gfx950") == 1
    assert ctx.rules == [(128, 2048, 3, 64)] and ctx.parts == 1
    ctx = _FakeCtx()
    autotune.apply(ctx, {"gfx950": {"16x1024xN3": {"tile_w": 128}}}, "gfx950")
    assert ctx.parts is None                     # no entry: the context keeps its split


class _CostCtx(_FakeCtx):
    def __init__(self):
        super().__init__()
        self.width = {}

    def set_tile_rule(self, H, W, N, tw):
        self.width[(H, W, N)] = tw


class _FakeTimer:
    """Plan time = 100 + per-shape cost of its tile width (weighted)."""
    shapes = [(16, 1024, 3), (128, 4096, 3)]
    cost = {(16, 1024, 3): {64: 3.0, 128: 2.0, 256: 2.03}, (128, 4096, 3): {64: 30.0, 128: 20.0, 256: 25.0}}

    def __init__(self, ctx):
        self.ctx = ctx

    def us_per_plan(self):
        return 100.0 + sum(self.cost[s][self.ctx.width.get(s, 64)] for s in self.shapes)


def test_refine_in_mix_keeps_only_clear_gains():
    ctx = _CostCtx()
    cache = {"gfx950": {"16x1024xN3": {"tile_w": 256}, "128x4096xN3": {"tile_w": 64}}}
    best = autotune.refine_in_mix(ctx, cache, "gfx950", _FakeTimer(ctx))
    # 128x4096: 64 -> 128 saves 10 of ~132 (kept); 16x1024: 256 -> 128 saves 0.03 (< 3 %, not kept)
    assert cache["gfx950"]["128x4096xN3"]["tile_w"] == 128
    assert cache["gfx950"]["16x1024xN3"]["tile_w"] == 256
    assert best == 100.0 + 2.03 + 20.0
    assert set(cache["gfx950"]["128x4096xN3"]["us_per_mixed_plan"]) == {"64", "128", "256"}
    assert ctx.width[(128, 4096, 3)] == 128
