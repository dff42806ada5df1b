"""The continuous-batching server on the GPU: every result served in the mix
equals (bit for bit) the same pair solved alone, both at the nominal load and
under overload, where pairs are batched and the captured graphs of every batch
size are replayed many times between eager copies."""
import math

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2212_00476_amd as zdt  # noqa: E402
from paper_2212_00476_amd import serving  # noqa: E402

_EX = {}


def note(msg):
    print(msg, flush=True)


def _executor():
    if "ex" not in _EX:
        note("building the pair pools and lanes")
        pairs = serving.make_pairs({"640x192_d64": 3, "1280x384_d128": 2, "1920x1080_d256": 1})
        _EX["ex"] = serving.GpuExecutor(pairs, vol_dtype=zdt.ZDT_F16, lanes=2,
                                        max_batch={"640x192_d64": 6, "1280x384_d128": 4, "1920x1080_d256": 2})
        _EX["npairs"] = {k: len(v) for k, v in pairs.items()}
    return _EX["ex"], _EX["npairs"]


@pytest.mark.parametrize("rate,duration", [(300.0, 1.5), (3000.0, 0.3)], ids=["nominal", "overload"])
def test_served_results_equal_alone(rate, duration):
    ex, npairs = _executor()
    reqs = serving.poisson_arrivals(rate, duration, serving.MIX, npairs, seed=11)
    note(f"serving {len(reqs)} requests at {rate}/s")
    serving.serve(reqs, ex.scheduler(), ex)
    st = serving.summarize(reqs)
    note(f"  {st}")
    assert st["completed"] == len(reqs)
    assert st["checked"] == len(reqs) and st["mismatched"] == 0
    assert all(r.t_arrive <= r.t_start <= r.t_done for r in reqs)
    assert all(not math.isnan(r.latency) for r in reqs)


def test_overload_batches_several_pairs():
    ex, npairs = _executor()
    reqs = [serving.Request(i, "640x192_d64", i % npairs["640x192_d64"], 0.0) for i in range(40)]
    sched = ex.scheduler()
    seen = []
    orig = ex.launch

    def launch(lane, batch):
        seen.append(len(batch))
        orig(lane, batch)
    ex.launch = launch
    try:
        serving.serve(reqs, sched, ex)
    finally:
        ex.launch = orig
    assert max(seen) == 6 and sum(seen) == 40
    assert all(r.ok for r in reqs)
