"""Serving scheduler on the CPU: admission by HBM budget, slots, continuous
batching and latency accounting, driven by a scripted executor on a virtual
clock (no GPU, deterministic)."""
import numpy as np
import pytest

from paper_1302_0435_amd.serve import ScriptedExecutor, Scheduler, request_bytes


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def run(arrivals, sizes, duration, budget, max_batch=64, slots=2, d=4, k=8):
    clk = VClock()
    ex = ScriptedExecutor(duration, clock=clk)
    sch = Scheduler(ex, np.asarray(sizes), d, k, budget, max_batch, slots)
    st = sch.run(np.asarray(arrivals, dtype=float), clock=clk, sleep=clk.sleep)
    return st, ex


def test_every_request_served_once_in_arrival_order():
    arrivals = np.cumsum(np.full(200, 0.001))
    st, ex = run(arrivals, [5] * 200, lambda c: 0.004, budget=1 << 30)
    assert np.all(~np.isnan(st.done_s))
    covered = []
    for first, count, _ in ex.submitted:
        covered.extend(range(first, first + count))
    assert covered == list(range(200))


def test_latency_is_measured_from_scheduled_arrival():
    arrivals = np.array([0.0, 0.5, 1.0])
    st, _ = run(arrivals, [3, 3, 3], lambda c: 0.010, budget=1 << 30)
    lat = st.latencies_ms()
    # alone in an idle system: latency = service time plus at most one poll step
    assert np.all(lat >= 10.0 - 1e-9) and np.all(lat <= 10.2)


def test_continuous_batching_packs_waiting_requests():
    # 100 requests arrive in 1 ms while two slots are busy for 50 ms each
    arrivals = np.linspace(0.0, 0.001, 100)
    st, ex = run(arrivals, [4] * 100, lambda c: 0.050, budget=1 << 30, max_batch=64, slots=2)
    sizes = [c for _, c, _ in ex.submitted]
    assert sum(sizes) == 100
    assert max(sizes) > 1            # later arrivals were batched together
    assert len(sizes) < 100


def test_budget_limits_bytes_in_flight():
    d, k = 4, 8
    one = request_bytes(10, d, k)
    arrivals = np.zeros(12)
    st, ex = run(arrivals, [10] * 12, lambda c: 0.01, budget=3 * one, max_batch=64, slots=4, d=d, k=k)
    assert all(c <= 3 for _, c, _ in ex.submitted)
    assert np.all(~np.isnan(st.done_s))


def test_budget_below_one_request_queues_without_crashing():
    d, k = 4, 8
    arrivals = np.array([0.0, 0.001])
    st, ex = run(arrivals, [10, 10], lambda c: 0.01, budget=request_bytes(10, d, k) - 1, d=d, k=k)
    assert ex.submitted == []
    assert np.all(np.isnan(st.done_s))
    assert st.summary(k)["completed"] == 0


def test_overload_grows_the_queue_but_serves_everyone():
    # service 20 ms per batch of <= 8, arrivals every 1 ms: over capacity
    arrivals = np.cumsum(np.full(400, 0.001))
    st, _ = run(arrivals, [6] * 400, lambda c: 0.020, budget=1 << 30, max_batch=8, slots=1)
    lat = st.latencies_ms()
    assert lat.size == 400
    assert st.max_queue > 100
    assert lat[-10:].mean() > 10 * lat[:10].mean()


@pytest.mark.parametrize("slots", [1, 3])
def test_slots_bound_concurrency(slots):
    arrivals = np.zeros(50)
    st, ex = run(arrivals, [5] * 50, lambda c: 0.01, budget=1 << 30, max_batch=5, slots=slots)
    assert sorted({s for _, _, s in ex.submitted}) == list(range(slots))
    assert np.all(~np.isnan(st.done_s))


class SlowStartExecutor(ScriptedExecutor):
    """An executor whose start takes `lag` seconds (like a device
    synchronisation) before its own time origin."""

    def __init__(self, duration, clock, lag):
        super().__init__(duration, clock=clock)
        self.lag = lag

    def start(self, clock=None):
        self.clock.sleep(self.lag)
        return super().start(clock)


def test_completions_are_placed_on_the_arrival_clock():
    # requests arrive at 0 and 0.1 s; the executor's origin lies 5 ms after
    # the loop's t0, so the first request waits for it and completes at
    # 5 + 10 ms, the second at 100 + 10 ms (plus at most one poll step)
    clk = VClock()
    ex = SlowStartExecutor(lambda c: 0.010, clk, 0.005)
    sch = Scheduler(ex, np.array([3, 3]), 4, 8, 1 << 30, 64, 2)
    st = sch.run(np.array([0.0, 0.1]), clock=clk, sleep=clk.sleep)
    lat = st.latencies_ms()
    assert 15.0 - 1e-9 <= lat[0] <= 15.2
    assert 10.0 - 1e-9 <= lat[1] <= 10.2


def test_warm_up_leaves_the_measured_run_unchanged():
    """The warm-up serves a burst and the head of the schedule on the same
    scheduler; the measured run that follows is the one a fresh scheduler
    gives (the scheduler keeps no state between runs)."""
    from paper_1302_0435_amd.serve import warm_up
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1e-3, size=300))
    sizes = rng.integers(4, 65, size=300)
    dur = lambda c: 0.002 + 1e-4 * c
    fresh, _ = run(arrivals, sizes, dur, budget=1 << 30)
    clk = VClock()
    ex = ScriptedExecutor(dur, clock=clk)
    sch = Scheduler(ex, sizes, 4, 8, 1 << 30, 64, 2)
    warm_up(sch, arrivals, burst=100, seconds=0.05, clock=clk, sleep=clk.sleep)
    first = [sub for sub in ex.submitted]
    assert sum(c for _, c, _ in first) == 100 + int((arrivals < 0.05).sum())
    clk.t = 0.0      # the same clock phase as the fresh run's
    st = sch.run(arrivals, clock=clk, sleep=clk.sleep)
    np.testing.assert_allclose(st.latencies_ms(), fresh.latencies_ms(), rtol=0, atol=1e-6)


def test_arena_first_fit_and_merging():
    from paper_1302_0435_amd.serve import Arena, BATCH_EXTRA
    a = Arena(4096, align=256)
    assert a.need(1) == 256 and a.need(256 - BATCH_EXTRA) == 256 and a.need(256) == 512
    x = a.alloc(1024); y = a.alloc(1024); z = a.alloc(2048)
    assert (x, y, z) == (0, 1024, 2048) and a.largest() == 0 and a.alloc(256) is None
    a.release(y, 1024)                     # a hole in the middle
    assert a.largest() == 1024 and a.alloc(2048) is None
    a.release(x, 1024)                     # merges with the hole
    assert a.free == [(0, 2048)]
    a.release(z, 2048)
    assert a.free == [(0, 4096)]


def test_in_flight_batches_hold_disjoint_ranges_of_the_budget():
    """The budget is one buffer: batches in flight at the same time hold
    disjoint ranges of it, each large enough for its requests."""
    from paper_1302_0435_amd.serve import BATCH_EXTRA
    rng = np.random.default_rng(11)
    d, k = 8, 16
    sizes = rng.integers(1, 65, size=400)
    arrivals = np.cumsum(rng.exponential(2e-4, size=400))
    budget = 5 * request_bytes(64, d, k) + 1000
    clk = VClock()
    ex = ScriptedExecutor(lambda c: 0.001 + 2e-4 * c, clock=clk)
    held = []
    orig = ex.submit

    def submit(b):
        orig(b)
        held.append(b)
    ex.submit = submit
    sch = Scheduler(ex, sizes, d, k, budget, 64, 3)
    st = sch.run(arrivals, clock=clk, sleep=clk.sleep)
    assert np.all(~np.isnan(st.done_s))
    spans = []
    for b in held:
        fp = sum(request_bytes(int(t), d, k) for t in sizes[b.first:b.first + b.count])
        assert b.nbytes == fp and b.arena_len >= fp + BATCH_EXTRA
        assert 0 <= b.arena_off and b.arena_off + b.arena_len <= budget
        spans.append((b.submit_s, b.submit_s + 0.001 + 2e-4 * b.count, b.arena_off, b.arena_off + b.arena_len))
    for i in range(len(spans)):
        for j in range(i + 1, len(spans)):
            t0, t1, a0, a1 = spans[i]
            u0, u1, c0, c1 = spans[j]
            if t0 < u1 and u0 < t1:          # in flight together
                assert a1 <= c0 or c1 <= a0
    assert max(b.count for b in held) > 1
