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


def test_scheduler_fifo_batches_and_lanes():
    s = Scheduler({"a": 1, "b": 2}, {"a": 3, "b": 2})
    for i, (shape, t) in enumerate([("a", 0.0), ("b", 0.1), ("a", 0.2), ("a", 0.3), ("a", 0.4), ("b", 0.5)]):
        s.arrive(Request(i, shape, 0, t))
    out = s.dispatch()
    # oldest waiting shape first; "a" gets its one lane with 3 requests in order,
    # "b" fills one lane with both of its requests
    assert [(lane, [r.rid for r in b]) for lane, b in out] == [(("a", 0), [0, 2, 3]), (("b", 0), [1, 5])]
    assert s.waiting() == 1 and s.dispatch() == []          # "a" has no free lane
    assert [r.rid for r in s.complete(("a", 0))] == [0, 2, 3]
    out = s.dispatch()
    assert [(lane, [r.rid for r in b]) for lane, b in out] == [(("a", 0), [4])]
    s.complete(("a", 0))
    s.complete(("b", 0))
    assert s.idle()


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-5)


class SimDevice:
    """A lane finishes a batch of n after base + per_pair * n seconds."""

    def __init__(self, clock, base, per_pair):
        self.clock, self.base, self.per_pair = clock, base, per_pair
        self.end, self.batches = {}, []

    def launch(self, lane, batch):
        self.clock.t += 2e-6                       # host cost of a launch
        self.end[lane] = self.clock.t + self.base[lane[0]] + self.per_pair[lane[0]] * len(batch)
        self.batches.append((lane, [r.rid for r in batch]))

    def poll(self, lane):
        return self.clock.t >= self.end[lane]

    def finish(self, lane, batch):
        for r in batch:
            r.ok = True


def test_serve_light_load_runs_pairs_alone():
    clk = SimClock()
    dev = SimDevice(clk, {"s": 1e-3}, {"s": 1e-3})
    reqs = [Request(i, "s", 0, 0.05 * i) for i in range(20)]     # 20 / s, service 2 ms
    serve(reqs, Scheduler({"s": 1}, {"s": 8}), dev, clock=clk, sleep=clk.sleep)
    assert all(len(b) == 1 for _, b in dev.batches)
    lat = np.array([r.latency for r in reqs])
    assert np.all(lat >= 2e-3) and np.all(lat < 2.5e-3)
    st = summarize(reqs)
    assert st["completed"] == 20 and st["mismatched"] == 0 and st["checked"] == 20


def test_serve_admits_arrivals_while_busy():
    """Under overload, requests that arrive while a lane runs are admitted
    together when it frees up, and the other lane of the shape overlaps."""
    clk = SimClock()
    # "s": 667 requests/s offered, two lanes of 8 pairs per 28 ms = 571/s: saturated
    dev = SimDevice(clk, {"s": 2e-2, "t": 1e-3}, {"s": 1e-3, "t": 1e-4})
    reqs = [Request(i, "s" if i % 3 else "t", 0, 1e-3 * i) for i in range(300)]   # 1000 / s
    serve(reqs, Scheduler({"s": 2, "t": 1}, {"s": 8, "t": 4}), dev, clock=clk, sleep=clk.sleep)
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


def test_budget_check_before_any_allocation():
    pytest.importorskip("torch")
    import paper_2212_00476_amd as zdt
    zdt.load()
    pairs = {"1920x1080_d256": [None]}
    with pytest.raises(ValueError, match="budget"):
        serving.GpuExecutor(pairs, lanes=4, max_batch={"1920x1080_d256": 8}, budget_bytes=16 << 30)
