"""The continuous-batching server on the GPU: every result served in the mix
equals (bit for bit) the same pair solved alone -- at the nominal load and
under overload, with a shape the server has not seen before, and under an HBM
budget tight enough that requests wait for memory and lanes are released and
reopened -- while the library-captured graphs of every batch size are
replayed many times between eager copies."""
import math

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2212_00476_amd as zdt  # noqa: E402
from paper_2212_00476_amd import serving  # noqa: E402

_POOLS = {}
MIX4 = {"640x192_d64": 0.45, "1280x384_d128": 0.35, "1920x1080_d256": 0.1, "320x96_d32": 0.1}


def note(msg):
    print(msg, flush=True)


def _pools():
    if not _POOLS:
        note("building the pair pools")
        shapes = serving.SHAPES + (serving.shape_of("320x96_d32"),)
        _POOLS.update(serving.make_pairs({"640x192_d64": 3, "1280x384_d128": 2, "1920x1080_d256": 1,
                                          "320x96_d32": 2}, shapes=shapes))
    return _POOLS


def _check_all(reqs):
    st = serving.summarize(reqs)
    note(f"  {st}")
    assert st["completed"] == len(reqs)
    assert st["checked"] == len(reqs) and st["mismatched"] == 0
    assert all(r.t_arrive <= r.t_start <= r.t_done for r in reqs)
    assert all(not math.isnan(r.latency) for r in reqs)
    # device-only time: positive, and within the end-to-end latency
    assert all(0.0 < r.device_ms <= 1e3 * r.latency for r in reqs)
    assert st["device_p50_ms"] <= st["p50_ms"] and st["device_p99_ms"] <= st["p99_ms"]
    return st


@pytest.mark.parametrize("rate,duration", [(300.0, 1.5), (3000.0, 0.3)], ids=["nominal", "overload"])
def test_served_results_equal_alone(rate, duration):
    pools = _pools()
    ex = serving.GpuExecutor(pools, vol_dtype=zdt.ZDT_F16)
    sched = ex.scheduler()
    reqs = serving.poisson_arrivals(rate, duration, MIX4, {k: len(v) for k, v in pools.items()}, seed=11)
    note(f"serving {len(reqs)} requests at {rate}/s")
    serving.serve(reqs, sched, ex)
    _check_all(reqs)
    assert ("320x96_d32", 0) in sched.lanes           # the shape seen for the first time got a lane
    assert ex.graph_captures >= len(sched.lanes)
    sched.close()


def test_tight_budget_waits_releases_and_reopens():
    """A 3 GB budget holds one 1920x1080 lane, one 1280x384 lane and a few
    small ones: under overload requests wait for memory and idle lanes of
    other shapes are released, and every result still equals the pair alone."""
    pools = _pools()
    ex = serving.GpuExecutor(pools, vol_dtype=zdt.ZDT_F16, budget_bytes=3 << 30)
    sched = ex.scheduler()
    reqs = serving.poisson_arrivals(3000.0, 0.3, MIX4, {k: len(v) for k, v in pools.items()}, seed=12)
    note(f"serving {len(reqs)} requests under a 3 GB budget")
    serving.serve(reqs, sched, ex)
    _check_all(reqs)
    note(f"  peak {sched.peak / 1e9:.2f} GB, waited for memory {len(sched.waited_for_memory)}, "
         f"lanes released {sched.released}")
    assert sched.peak <= 3 << 30
    assert sched.waited_for_memory and sched.released > 0
    sched.close()


def test_overload_batches_several_pairs():
    pools = _pools()
    ex = serving.GpuExecutor(pools, vol_dtype=zdt.ZDT_F16)
    n = len(pools["640x192_d64"])
    reqs = [serving.Request(i, "640x192_d64", i % n, 0.0) for i in range(40)]
    sched = ex.scheduler()
    seen = []
    orig = ex.launch

    def launch(lane, batch):
        seen.append(len(batch))
        orig(lane, batch)
    ex.launch = launch
    serving.serve(reqs, sched, ex)
    cap, _ = ex.lane_plan("640x192_d64")
    assert max(seen) == cap and sum(seen) == 40
    assert all(r.ok for r in reqs)
    sched.close()


def test_library_graph_replays_equal_eager_solves():
    """zdt_graph_create captures a batch; replays after refilling the images
    give the same disparities as eager solves of the new images."""
    pools = _pools()
    prs = pools["640x192_d64"]
    p = zdt.params(640, 192, 64, vol_dtype=zdt.ZDT_F16)
    H, W = 192, 640
    left = torch.empty((2, H, W), dtype=torch.uint8, device="cuda")
    right = torch.empty_like(left)
    disp = torch.empty((2, H, W), dtype=torch.int32, device="cuda")
    vols = [torch.empty(zdt.volume_size(p), dtype=torch.uint8, device="cuda") for _ in range(2)]
    wss = [torch.empty(zdt.workspace_size(p), dtype=torch.uint8, device="cuda") for _ in range(2)]
    jobs = [(p, left[i], right[i], disp[i], vols[i], wss[i]) for i in range(2)]
    s = torch.cuda.Stream()
    for k in range(3):
        for i in range(2):
            pr = prs[(k + i) % len(prs)]
            left[i].copy_(torch.from_numpy(pr.left))
            right[i].copy_(torch.from_numpy(pr.right))
        torch.cuda.synchronize()
        if k == 0:
            g = zdt.Graph(jobs, s)                # runs the batch once, eagerly, then records it
        else:
            g.launch(s)
        s.synchronize()
        got = disp.clone()
        for i in range(2):
            alone = torch.empty((H, W), dtype=torch.int32, device="cuda")
            zdt.stereo_solve(p, left[i], right[i], alone, vols[i], wss[i])
            torch.cuda.synchronize()
            assert torch.equal(got[i], alone), (k, i)
    g.close()
