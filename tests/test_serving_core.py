"""Serving-loop logic on the CPU: a fake device backend and a fake clock.

Checks admission against the HBM budget, FIFO order per sensor, slot reuse
and backpressure, continuous batching across streams, and the latency
order statistics."""
import math

import pytest

from paper_2003_00575_amd.serve import (BudgetError, ServingCore, SensorSpec, order_stat,
                                        poisson_schedule)


class FakeClock:
    """Advances by `tick` on every read, so busy-polling loops make progress."""

    def __init__(self, tick=1e-5):
        self.t = 0.0
        self.tick = tick

    def __call__(self):
        self.t += self.tick
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Each launch takes `cost_per_frame * frames + fixed` seconds of fake time."""

    def __init__(self, clock, fixed=1e-3, per_frame=1e-4):
        self.clock, self.fixed, self.per_frame = clock, fixed, per_frame
        self.registered, self.staged, self.launches = [], [], []

    def sensor_bytes(self, spec):
        return 1000

    def scratch_bytes(self, px):
        return px

    def register(self, spec, n):
        self.registered.append((spec.sensor, n))

    def stage(self, sensor, slot, frame):
        self.staged.append((sensor, slot, frame))

    def launch(self, stream, items):
        end = self.clock() + self.fixed + self.per_frame * len(items)
        self.launches.append((stream, list(items)))
        return end

    def done(self, token):
        return self.clock() >= token


def test_order_statistics_are_exact():
    xs = list(range(1, 101))
    assert order_stat(xs, 0.5) == 50
    assert order_stat(xs, 0.99) == 99
    assert order_stat([7.0], 0.99) == 7.0
    assert math.isnan(order_stat([], 0.5))


def test_admission_by_budget():
    clk = FakeClock()
    be = FakeBackend(clk)
    spec = SensorSpec(0, 16, 1024, 3, 0.5)
    per_sensor = 1000 + 2 * spec.frame_bytes
    core = ServingCore(be, hbm_budget=3 * per_sensor + 3 * 2 * 16 * 1024 + 10, n_streams=3,
                       max_batch=2, slots_per_sensor=2, clock=clk)
    for s in range(3):
        core.add_sensor(SensorSpec(s, 16, 1024, 3, 0.5))
    with pytest.raises(BudgetError):
        core.add_sensor(SensorSpec(3, 16, 1024, 3, 0.5))
    assert [r[0] for r in be.registered] == [0, 1, 2]
    assert 3 not in core.specs


def test_fifo_backpressure_and_batching():
    clk = FakeClock()
    be = FakeBackend(clk, fixed=5e-3, per_frame=0.0)
    core = ServingCore(be, hbm_budget=1 << 40, n_streams=1, max_batch=8, slots_per_sensor=2,
                       max_queue=3, clock=clk)
    core.add_sensor(SensorSpec(0, 16, 1024, 3, 0.5))
    for f in range(6):
        core.arrive(0, f, clk())
    # two slots: frames 0, 1 admitted; queue holds 3 of the remaining 4 (oldest dropped)
    assert [st[2] for st in be.staged] == [0, 1]
    assert core.dropped == 1
    assert [r.frame for r in core.waiting[0]] == [3, 4, 5]
    assert core.launch_ready() == 2
    assert core.launch_ready() == 0            # the only stream is busy
    clk.t += 6e-3
    assert core.poll() == 2
    # freed slots admit the next frames in arrival order
    assert [st[2] for st in be.staged] == [0, 1, 3, 4]
    core.launch_ready()
    clk.t += 6e-3
    core.poll()
    core.launch_ready()
    clk.t += 6e-3
    core.poll()
    assert not core.busy()
    done = sorted(r.frame for r in core.records if math.isfinite(r.t_done))
    assert done == [0, 1, 3, 4, 5]


def test_continuous_batching_uses_idle_streams():
    clk = FakeClock()
    be = FakeBackend(clk, fixed=2e-3, per_frame=1e-4)
    core = ServingCore(be, hbm_budget=1 << 40, n_streams=2, max_batch=4, slots_per_sensor=4,
                       clock=clk)
    for s in range(4):
        core.add_sensor(SensorSpec(s, 32, 1800, 3, 0.5))
    sched = poisson_schedule([200.0] * 4, 0.5, seed=3)
    core.run(sched, sleep=clk.sleep)
    st = core.stats()
    assert st["frames"] == len(sched) and st["dropped"] == 0
    used_streams = {stream for stream, _ in be.launches}
    assert used_streams == {0, 1}
    assert max(len(items) for _, items in be.launches) > 1      # batching happened
    # every launch holds frames that were admitted before it
    for r in core.records:
        assert r.t_arrival <= r.t_admit <= r.t_launch <= r.t_done
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_poisson_schedule_rates():
    sched = poisson_schedule([10.0, 20.0], 200.0, seed=1)
    n0 = sum(1 for _, s, _ in sched if s == 0)
    n1 = sum(1 for _, s, _ in sched if s == 1)
    assert abs(n0 / 200.0 - 10.0) < 1.0 and abs(n1 / 200.0 - 20.0) < 1.5
    assert all(a[0] <= b[0] for a, b in zip(sched, sched[1:]))
    fast = poisson_schedule([10.0], 10.0, seed=1, speedup=4.0)
    assert abs(len(fast) / 10.0 - 40.0) < 8.0
