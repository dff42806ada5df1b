"""Continuous-batching stereo server on one GPU.

Requests (a stereo pair of one of several shapes) arrive over time; each shape
has a few execution lanes, every lane with its own HIP stream, its own
device-resident inputs, working volumes, workspaces and disparity buffers for
up to `max_batch` pairs, and one captured HIP graph per batch size.  Whenever a
lane is free and pairs of its shape are waiting, the lane takes up to
`max_batch` of them (oldest first): their images are copied into the lane's
slots, the graph for that batch size is replayed (one launch per stage over
all of them, see ``stereo_solve_batch``) and the disparities are copied back
to pinned host memory.  Pairs that arrive while others run are admitted as soon
as a lane of their shape frees up, and lanes of different shapes (and of the
same shape) overlap on the device.  The lanes' volumes are allocated once, up
front, and must fit the HBM budget for live cost volumes.

The paper solves one pair at a time without streams; this module is the
serving layer around its hot path.  The scheduler is plain host logic
(``Scheduler``, ``serve``) driven by an executor; ``GpuExecutor`` runs it on
the device and can check every result against the same pair solved alone.

    python -m paper_2212_00476_amd.serving --rate 300 --duration 10
"""
from __future__ import annotations

import argparse
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Shape:
    name: str
    W: int
    H: int
    D: int


SHAPES = (Shape("640x192_d64", 640, 192, 64), Shape("1280x384_d128", 1280, 384, 128),
          Shape("1920x1080_d256", 1920, 1080, 256))
MIX = {"640x192_d64": 0.5, "1280x384_d128": 0.4, "1920x1080_d256": 0.1}


@dataclass
class Request:
    rid: int
    shape: str
    pair: int          # index into the shape's pool of input pairs
    t_arrive: float    # seconds after the start of the run
    t_start: float = math.nan
    t_done: float = math.nan
    ok: bool | None = None   # result equal to the pair solved alone (when checked)

    @property
    def latency(self):
        return self.t_done - self.t_arrive


def poisson_arrivals(rate, duration, mix=MIX, pairs_per_shape=None, seed=0):
    """Requests of a Poisson process of the given rate over [0, duration): each
    picks a shape with the mix's probabilities and one of the shape's pairs."""
    # independent streams: the times and shapes do not depend on the pool sizes
    r_t, r_s, r_p = (np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3))
    names = list(mix)
    prob = np.array([mix[n] for n in names], np.float64)
    prob /= prob.sum()
    out, t = [], 0.0
    while True:
        t += r_t.exponential(1.0 / rate)
        if t >= duration:
            return out
        name = names[int(r_s.choice(len(names), p=prob))]
        npairs = 1 if pairs_per_shape is None else pairs_per_shape[name]
        out.append(Request(len(out), name, int(r_p.uniform() * npairs), t))


class Scheduler:
    """Per-shape FIFO queues and execution lanes.  A lane is (shape, k)."""

    def __init__(self, lanes, max_batch):
        self.max_batch = dict(max_batch)
        self.queues = {s: deque() for s in lanes}
        self.free = {s: deque((s, k) for k in range(n)) for s, n in lanes.items()}
        self.running = {}

    def arrive(self, req):
        self.queues[req.shape].append(req)

    def dispatch(self):
        """[(lane, batch)] for every free lane whose shape has waiting requests;
        shapes whose oldest request waited longest go first."""
        out = []
        order = sorted((q[0].t_arrive, s) for s, q in self.queues.items() if q)
        for _, s in order:
            q, free = self.queues[s], self.free[s]
            while q and free:
                lane = free.popleft()
                batch = [q.popleft() for _ in range(min(len(q), self.max_batch[s]))]
                self.running[lane] = batch
                out.append((lane, batch))
        return out

    def complete(self, lane):
        batch = self.running.pop(lane)
        self.free[lane[0]].append(lane)
        return batch

    def busy_lanes(self):
        return list(self.running)

    def waiting(self):
        return sum(len(q) for q in self.queues.values())

    def idle(self):
        return not self.running and self.waiting() == 0


def serve(requests, scheduler, executor, clock=time.perf_counter, sleep=time.sleep):
    """Run the requests in real time (request i arrives t_arrive seconds after
    the start) and return them with t_start / t_done filled in."""
    reqs = sorted(requests, key=lambda r: r.t_arrive)
    t0 = clock()
    i = 0
    while i < len(reqs) or not scheduler.idle():
        now = clock() - t0
        while i < len(reqs) and reqs[i].t_arrive <= now:
            scheduler.arrive(reqs[i])
            i += 1
        progressed = False
        for lane in scheduler.busy_lanes():
            if executor.poll(lane):
                t = clock() - t0
                batch = scheduler.complete(lane)
                for r in batch:
                    r.t_done = t
                executor.finish(lane, batch)
                progressed = True
        for lane, batch in scheduler.dispatch():
            t = clock() - t0
            for r in batch:
                r.t_start = t
            executor.launch(lane, batch)
            progressed = True
        if not progressed:
            nxt = reqs[i].t_arrive - (clock() - t0) if i < len(reqs) else 0.0
            sleep(min(max(nxt, 0.0), 2e-4) if scheduler.busy_lanes() or nxt > 0 else 0.0)
    return reqs


def summarize(reqs, duration=None):
    done = [r for r in reqs if not math.isnan(r.t_done)]
    lat = np.array([r.latency for r in done]) * 1e3
    span = duration if duration is not None else (max(r.t_done for r in done) - min(r.t_arrive for r in done))
    out = {"requests": len(reqs), "completed": len(done), "pairs_per_s": round(len(done) / span, 2) if span else None,
           "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
           "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
           "checked": sum(r.ok is not None for r in done), "mismatched": sum(r.ok is False for r in done)}
    per = {}
    for s in sorted({r.shape for r in done}):
        ls = np.array([r.latency for r in done if r.shape == s]) * 1e3
        per[s] = {"n": int(len(ls)), "p50_ms": round(float(np.percentile(ls, 50)), 3),
                  "p99_ms": round(float(np.percentile(ls, 99)), 3)}
    out["per_shape"] = per
    return out


@dataclass
class _Lane:
    shape: Shape
    stream: object
    left: object            # uint8 [B][H][W] on the device (slot k = [k])
    right: object
    disp: object            # int32 [B][H][W] on the device
    host_out: object        # int32 [B][H][W], pinned
    vols: list
    wss: list
    jobs: list
    event: object
    graphs: dict = field(default_factory=dict)
    batch: list = field(default_factory=list)


class GpuExecutor:
    """Lanes on the device: buffers allocated once, one captured graph per
    (lane, batch size), a completion event per launch.

    pairs: {shape name: [StereoPair, ...]} -- the inputs requests refer to.
    check: compare every result with the pair solved alone (bit for bit)."""

    def __init__(self, pairs, shapes=SHAPES, vol_dtype=None, lanes=2, max_batch=None, budget_bytes=64 << 30,
                 radius=4, sigma_s=20.0, sigma_r=0.1, dt_iters=3, graphs=True, check=True, device="cuda"):
        import torch

        from . import _lib as lib
        self.torch, self.lib = torch, lib
        vol_dtype = lib.ZDT_F16 if vol_dtype is None else vol_dtype
        self.shapes = {s.name: s for s in shapes if s.name in pairs}
        max_batch = max_batch or {"640x192_d64": 8, "1280x384_d128": 8, "1920x1080_d256": 2}
        self.max_batch = {s: max_batch.get(s, 4) for s in self.shapes}
        self.nlanes = {s: (lanes[s] if isinstance(lanes, dict) else lanes) for s in self.shapes}
        self.params = {s: lib.params(sh.W, sh.H, sh.D, radius, sigma_s, sigma_r, dt_iters, vol_dtype)
                       for s, sh in self.shapes.items()}
        vol_bytes = sum(self.nlanes[s] * self.max_batch[s] * lib.volume_size(self.params[s]) for s in self.shapes)
        if vol_bytes > budget_bytes:
            raise ValueError("lanes need %.2f GB of cost volumes, over the %.2f GB budget"
                             % (vol_bytes / 1e9, budget_bytes / 1e9))
        self.volume_bytes = vol_bytes
        dev = torch.device(device)
        self.pinned = {s: [(torch.from_numpy(p.left).pin_memory(), torch.from_numpy(p.right).pin_memory())
                           for p in pairs[s]] for s in self.shapes}
        vt = {lib.ZDT_F32: torch.float32, lib.ZDT_F16: torch.float16, lib.ZDT_BF16: torch.bfloat16}[vol_dtype]
        self.lanes = {}
        for s, sh in self.shapes.items():
            p, B = self.params[s], self.max_batch[s]
            wsz = lib.workspace_size(p)
            for k in range(self.nlanes[s]):
                u8 = dict(dtype=torch.uint8, device=dev)
                left, right = torch.empty((B, sh.H, sh.W), **u8), torch.empty((B, sh.H, sh.W), **u8)
                disp = torch.empty((B, sh.H, sh.W), dtype=torch.int32, device=dev)
                vols = [torch.empty((sh.H, sh.W, sh.D), dtype=vt, device=dev) for _ in range(B)]
                wss = [torch.empty(wsz, **u8) if wsz else None for _ in range(B)]
                jobs = [(p, left[i], right[i], disp[i], vols[i], wss[i]) for i in range(B)]
                host_out = torch.empty((B, sh.H, sh.W), dtype=torch.int32).pin_memory()
                self.lanes[(s, k)] = _Lane(sh, torch.cuda.Stream(device=dev), left, right, disp, host_out, vols, wss,
                                           jobs, torch.cuda.Event())
        self.use_graphs = graphs
        self.check = check
        self.alone = {}
        if check:
            for s in self.shapes:
                self.alone[s] = [self._solve_alone(s, i) for i in range(len(self.pinned[s]))]
        if graphs:
            self._capture()

    def _solve_alone(self, s, i):
        torch, lib, sh = self.torch, self.lib, self.shapes[s]
        p = self.params[s]
        left, right = (t.cuda() for t in self.pinned[s][i])
        disp = torch.empty((sh.H, sh.W), dtype=torch.int32, device="cuda")
        vol = torch.empty(lib.volume_size(p), dtype=torch.uint8, device="cuda")
        wsz = lib.workspace_size(p)
        ws = torch.empty(wsz, dtype=torch.uint8, device="cuda") if wsz else None
        lib.stereo_solve(p, left, right, disp, vol, ws)
        out = disp.cpu().numpy()
        del vol, ws
        return out

    def _capture(self):
        torch, lib = self.torch, self.lib
        for lane in self.lanes.values():
            for n in range(1, self.max_batch[lane.shape.name] + 1):
                with torch.cuda.stream(lane.stream):     # warm-up outside the capture
                    lib.stereo_solve_batch(lane.jobs[:n], stream=lane.stream)
                lane.stream.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=lane.stream):
                    lib.stereo_solve_batch(lane.jobs[:n], stream=torch.cuda.current_stream())
                lane.graphs[n] = g
        torch.cuda.synchronize()

    def launch(self, lane_id, batch):
        torch, lane = self.torch, self.lanes[lane_id]
        n = len(batch)
        with torch.cuda.stream(lane.stream):
            for k, r in enumerate(batch):
                src_l, src_r = self.pinned[r.shape][r.pair]
                lane.left[k].copy_(src_l, non_blocking=True)
                lane.right[k].copy_(src_r, non_blocking=True)
            if self.use_graphs:
                lane.graphs[n].replay()
            else:
                self.lib.stereo_solve_batch(lane.jobs[:n], stream=lane.stream)
            lane.host_out[:n].copy_(lane.disp[:n], non_blocking=True)
            lane.event.record(lane.stream)
        lane.batch = batch

    def poll(self, lane_id):
        return self.lanes[lane_id].event.query()

    def finish(self, lane_id, batch):
        if not self.check:
            return
        lane = self.lanes[lane_id]
        for k, r in enumerate(batch):
            r.ok = bool(np.array_equal(lane.host_out[k].numpy(), self.alone[r.shape][r.pair]))

    def scheduler(self):
        return Scheduler(self.nlanes, self.max_batch)


def per_pair_capacity(reqs, pairs, vol_dtype, radius=4, sigma_s=20.0, sigma_r=0.1, dt_iters=3):
    """Pairs per second of the plain form: the same requests solved one at a
    time on one stream (upload, stereo_solve, download), no batching, no graphs."""
    import torch

    from . import _lib as lib
    bufs = {}
    for name in {r.shape for r in reqs}:
        sh = next(s for s in SHAPES if s.name == name)
        p = lib.params(sh.W, sh.H, sh.D, radius, sigma_s, sigma_r, dt_iters, vol_dtype)
        wsz = lib.workspace_size(p)
        bufs[name] = (p, torch.empty((sh.H, sh.W), dtype=torch.uint8, device="cuda"),
                      torch.empty((sh.H, sh.W), dtype=torch.uint8, device="cuda"),
                      torch.empty((sh.H, sh.W), dtype=torch.int32, device="cuda"),
                      torch.empty(lib.volume_size(p), dtype=torch.uint8, device="cuda"),
                      torch.empty(wsz, dtype=torch.uint8, device="cuda") if wsz else None,
                      torch.empty((sh.H, sh.W), dtype=torch.int32).pin_memory())
    pinned = {k: [(torch.from_numpy(q.left).pin_memory(), torch.from_numpy(q.right).pin_memory()) for q in v]
              for k, v in pairs.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        p, left, right, disp, vol, ws, out = bufs[r.shape]
        left.copy_(pinned[r.shape][r.pair][0], non_blocking=True)
        right.copy_(pinned[r.shape][r.pair][1], non_blocking=True)
        lib.stereo_solve(p, left, right, disp, vol, ws)
        out.copy_(disp, non_blocking=True)
    torch.cuda.synchronize()
    return len(reqs) / (time.perf_counter() - t0)


def make_pairs(per_shape, shapes=SHAPES, seed=1000):
    """Input pools: `per_shape[name]` synthetic scenes of each shape."""
    from . import scenes
    return {s.name: [scenes.planes_pair(s.W, s.H, s.D, seed=seed + 17 * i + s.W) for i in range(per_shape[s.name])]
            for s in shapes if per_shape.get(s.name, 0) > 0}


def run(rate=300.0, duration=10.0, vol_dtype=None, pairs_per_shape=None, lanes=2, graphs=True, check=True, seed=0,
        autotune=True):
    """Serve a Poisson stream of the mixed shapes and summarise it."""
    from . import _lib as lib
    pairs_per_shape = pairs_per_shape or {"640x192_d64": 4, "1280x384_d128": 2, "1920x1080_d256": 1}
    pairs = make_pairs(pairs_per_shape)
    if autotune:
        vd = lib.ZDT_F16 if vol_dtype is None else vol_dtype
        for s in SHAPES:
            if s.name in pairs:
                lib.autotune(lib.params(s.W, s.H, s.D, vol_dtype=vd))
    ex = GpuExecutor(pairs, vol_dtype=vol_dtype, lanes=lanes, graphs=graphs, check=check)
    reqs = poisson_arrivals(rate, duration, MIX, {k: len(v) for k, v in pairs.items()}, seed=seed)
    serve(reqs, ex.scheduler(), ex)
    out = summarize(reqs)
    out.update({"offered_rate": rate, "duration_s": duration, "volume_gb": round(ex.volume_bytes / 1e9, 2),
                "graphs": graphs})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--rate", type=float, default=300.0)
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    print(json.dumps(run(args.rate, args.duration, graphs=not args.no_graphs, check=not args.no_check)))


if __name__ == "__main__":
    main()
