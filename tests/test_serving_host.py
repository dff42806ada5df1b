"""Host logic of the continuous-batching server, run against a simulated clock
and a simulated device (no GPU): arrivals, admission, batching, lane reuse,
latency accounting and the HBM budget check."""
import math

import numpy as np
import pytest

from paper_2212_00476_amd import serving
from paper_2212_00476_amd.serving import Request, Scheduler, poisson_arrivals, serve, summarize


def test_poisson_arrivals_rate_mix_and_seed():
    reqs = poisson_arrivals(300.0, 60.0, serving.MIX, {"640x192_d64": 4, "1280x384_d128": 2, "1920x1080_d256": 1},
                            seed=3)
    n = len(reqs)
    assert abs(n - 18000) < 4 * math.sqrt(18000)
    t = np.array([r.t_arrive for r in reqs])
    assert np.all(np.diff(t) > 0) and t[0] >= 0 and t[-1] < 60.0
    # exponential gaps: mean 1/rate, coefficient of variation ~ 1
    gaps = np.diff(t)
    assert abs(gaps.mean() * 300 - 1) < 0.03 and abs(gaps.std() / gaps.mean() - 1) < 0.05
    for name, frac in serving.MIX.items():
        got = sum(r.shape == name for r in reqs) / n
        assert abs(got - frac) < 0.02, (name, got)
    assert all(0 <= r.pair < {"640x192_d64": 4, "1280x384_d128": 2, "1920x1080_d256": 1}[r.shape] for r in reqs)
    again = poisson_arrivals(300.0, 60.0, serving.MIX, None, seed=3)
    assert [(r.t_arrive, r.shape) for r in again] == [(r.t_arrive, r.shape) for r in reqs]


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


class SimDevice:
    """Lanes of `cap[shape]` pairs costing `nbytes[shape]`; a lane finishes a
    batch of n after base + per_pair * n seconds."""

    def __init__(self, clock, base, per_pair, cap, nbytes):
        self.clock, self.base, self.per_pair, self.cap, self.nbytes = clock, base, per_pair, cap, nbytes
        self.end, self.batches, self.created, self.destroyed = {}, [], [], []
        self.live = set()

    def lane_plan(self, shape):
        return self.cap[shape], self.nbytes[shape]

    def create_lane(self, lane, shape, cap):
        assert lane not in self.live
        self.live.add(lane)
        self.created.append(lane)

    def destroy_lane(self, lane):
        self.live.remove(lane)
        self.destroyed.append(lane)

    def launch(self, lane, batch):
        assert lane in self.live
        self.clock.t += 2e-6                       # host cost of a launch
        self.end[lane] = self.clock.t + self.base[lane[0]] + self.per_pair[lane[0]] * len(batch)
        self.batches.append((lane, [r.rid for r in batch]))

    def poll(self, lane):
        return self.clock.t >= self.end[lane]

    def finish(self, lane, batch):
        for r in batch:
            r.ok = True


def _sim(base, per_pair, cap, nbytes, budget, max_lanes=4):
    clk = SimClock()
    dev = SimDevice(clk, base, per_pair, cap, nbytes)
    return clk, dev, Scheduler(dev, budget, max_lanes)


def test_scheduler_fifo_batches_and_lanes():
    _, dev, s = _sim({}, {}, {"a": 3, "b": 2}, {"a": 10, "b": 10}, budget=30, max_lanes=1)
    for i, (shape, t) in enumerate([("a", 0.0), ("b", 0.1), ("a", 0.2), ("a", 0.3), ("a", 0.4), ("b", 0.5)]):
        s.arrive(Request(i, shape, 0, t))
    out = s.dispatch()
    # oldest waiting shape first; lanes are opened on demand: "a" gets one with
    # 3 requests in order, "b" one with both of its requests
    assert [(lane, [r.rid for r in b]) for lane, b in out] == [(("a", 0), [0, 2, 3]), (("b", 0), [1, 5])]
    assert dev.created == [("a", 0), ("b", 0)] and s.used == 20
    assert s.waiting() == 1 and s.dispatch() == []          # "a" has its one lane busy
    assert [r.rid for r in s.complete(("a", 0))] == [0, 2, 3]
    out = s.dispatch()
    assert [(lane, [r.rid for r in b]) for lane, b in out] == [(("a", 0), [4])]
    s.complete(("a", 0))
    s.complete(("b", 0))
    assert s.idle() and not s.waited_for_memory


def test_unseen_shape_gets_a_lane_on_first_arrival():
    _, dev, s = _sim({}, {}, {"a": 2, "777x333_d48": 1}, {"a": 10, "777x333_d48": 7}, budget=100)
    s.arrive(Request(0, "777x333_d48", 0, 0.0))
    out = s.dispatch()
    assert out and out[0][0] == ("777x333_d48", 0) and dev.created == [("777x333_d48", 0)]
    assert s.used == 7


def test_over_budget_request_waits_until_memory_frees():
    """Budget for one big lane or two small ones: a big request arriving while
    both small lanes run waits (and keeps younger small requests from opening
    lanes), then takes the memory of the released small lanes."""
    _, dev, s = _sim({}, {}, {"small": 1, "big": 1}, {"small": 40, "big": 70}, budget=100)
    s.arrive(Request(0, "small", 0, 0.0))
    s.arrive(Request(1, "small", 0, 0.1))
    assert [lane for lane, _ in s.dispatch()] == [("small", 0), ("small", 1)]
    s.arrive(Request(2, "big", 0, 0.2))
    s.arrive(Request(3, "small", 0, 0.3))
    assert s.dispatch() == [] and s.waited_for_memory == {2}
    s.complete(("small", 0))
    # the small lane that freed up is released for the older big request, which
    # still does not fit; the younger small request may not open a lane
    assert s.dispatch() == [] and s.used == 40 and ("small", 0) in dev.destroyed
    s.complete(("small", 1))
    out = s.dispatch()
    assert [(lane, [r.rid for r in b]) for lane, b in out] == [(("big", 0), [2])]
    assert s.used == 70 and s.peak == 80
    s.complete(("big", 0))
    out = s.dispatch()                        # the big lane is released for the small one
    assert [(lane, [r.rid for r in b]) for lane, b in out] == [(("small", 2), [3])]


def test_a_lane_larger_than_the_budget_is_refused():
    _, _, s = _sim({}, {}, {"huge": 1}, {"huge": 1000}, budget=100)
    with pytest.raises(ValueError, match="budget"):
        s.arrive(Request(0, "huge", 0, 0.0))


def test_serve_light_load_runs_pairs_alone():
    clk, dev, sched = _sim({"s": 1e-3}, {"s": 1e-3}, {"s": 8}, {"s": 1}, budget=10, max_lanes=1)
    reqs = [Request(i, "s", 0, 0.05 * i) for i in range(20)]     # 20 / s, service 2 ms
    serve(reqs, sched, dev, clock=clk, sleep=clk.sleep)
    assert all(len(b) == 1 for _, b in dev.batches)
    lat = np.array([r.latency for r in reqs])
    assert np.all(lat >= 2e-3) and np.all(lat < 2.5e-3)
    st = summarize(reqs)
    assert st["completed"] == 20 and st["mismatched"] == 0 and st["checked"] == 20


def test_serve_admits_arrivals_while_busy():
    """Under overload, requests that arrive while a lane runs are admitted
    together when it frees up, and the other lane of the shape overlaps."""
    # "s": 667 requests/s offered, two lanes of 8 pairs per 28 ms = 571/s: saturated
    clk, dev, sched = _sim({"s": 2e-2, "t": 1e-3}, {"s": 1e-3, "t": 1e-4}, {"s": 8, "t": 4}, {"s": 1, "t": 1},
                           budget=3, max_lanes=2)
    reqs = [Request(i, "s" if i % 3 else "t", 0, 1e-3 * i) for i in range(300)]   # 1000 / s
    serve(reqs, sched, dev, clock=clk, sleep=clk.sleep)
    assert all(not math.isnan(r.t_done) for r in reqs)
    assert all(r.t_arrive <= r.t_start <= r.t_done for r in reqs)
    sizes = [len(b) for lane, b in dev.batches if lane[0] == "s"]
    assert max(sizes) == 8 and min(sizes) >= 1 and sum(sizes) == 200
    # both lanes of "s" were used and their batches overlapped in time
    assert {lane for lane, _ in dev.batches if lane[0] == "s"} == {("s", 0), ("s", 1)}
    # FIFO per shape: start order follows arrival order
    for shape in "st":
        starts = [r.t_start for r in sorted(reqs, key=lambda r: r.t_arrive) if r.shape == shape]
        assert starts == sorted(starts)
    st = summarize(reqs)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_serve_under_a_tight_budget_completes_every_request():
    """A mix whose lanes cannot all be resident: lanes are released and
    reopened as shapes alternate, every request completes, in FIFO order per
    shape, and the budget is never exceeded."""
    clk, dev, sched = _sim({"a": 2e-3, "b": 5e-3, "c": 1e-3}, {"a": 1e-4, "b": 1e-3, "c": 1e-4},
                           {"a": 4, "b": 1, "c": 8}, {"a": 30, "b": 60, "c": 20}, budget=90)
    rng = np.random.default_rng(4)
    reqs = [Request(i, str(rng.choice(["a", "b", "c"])), 0, 2e-4 * i) for i in range(400)]
    serve(reqs, sched, dev, clock=clk, sleep=clk.sleep)
    assert all(not math.isnan(r.t_done) for r in reqs)
    assert sched.peak <= 90 and sched.released > 0 and sched.waited_for_memory
    for shape in "abc":
        starts = [r.t_start for r in sorted(reqs, key=lambda r: r.t_arrive) if r.shape == shape]
        assert starts == sorted(starts)


def test_shape_names():
    sh = serving.shape_of("777x333_d48")
    assert (sh.W, sh.H, sh.D) == (777, 333, 48)
