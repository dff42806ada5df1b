"""Continuous-batching stereo server on one GPU.

Requests (a stereo pair of any size and disparity range) arrive over time.
Pairs of one shape (W, H, D) are served by *lanes*: a lane owns a HIP stream,
device buffers for up to B pairs of its shape (images, working volume,
workspace, disparities) and pinned host memory for the results, and replays a
library-captured HIP graph per batch size (``zdt_graph_create``).  Whenever a
lane is free and pairs of its shape wait, it takes up to B of them (oldest
first): their images are copied into its slots, the graph for that batch size
is replayed (one launch per stage over all of them, see
``stereo_solve_batch``) and the disparities are copied back.  Pairs that arrive
while others run are admitted as soon as a lane frees up, and lanes of
different shapes (and of the same shape) overlap on the device.

Admission is by an HBM budget for live buffers (64 GB by default): a lane is
created on demand -- for a shape seen for the first time, or when every lane
of a busy shape is taken -- only if its bytes (B pairs' volumes, workspaces,
images and disparities) fit in what the budget has left.  Otherwise idle lanes
of other shapes are released, least recently used first; if that is not
enough, the request waits until memory frees, and while the oldest waiting
request waits for memory no new lane is opened for a younger one.  A shape's
graphs are captured on its lanes' first batches of each size.

The paper solves one pair at a time without streams; this module is the
serving layer around its hot path.  The scheduler is plain host logic
(``Scheduler``, ``serve``) driven by an executor; ``GpuExecutor`` runs it on
the device and can check every result against the same pair solved alone.
Latency is reported end to end (arrival on the host to the disparities in
pinned host memory, uploads and downloads included) and device-only (the
kernels of the batch a request was solved in, timed with events on its lane's
stream).

    python -m paper_2212_00476_amd.serving --rate 300 --duration 60
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


def shape_of(name):
    """Shape named "<W>x<H>_d<D>"."""
    wh, d = name.split("_d")
    w, h = wh.split("x")
    return Shape(name, int(w), int(h), int(d))


SHAPES = (shape_of("640x192_d64"), shape_of("1280x384_d128"), shape_of("1920x1080_d256"))
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
    device_ms: float = math.nan   # device time of the batch it was solved in (kernels only)

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


@dataclass
class _LaneState:
    shape: str
    capacity: int      # pairs per batch
    nbytes: int
    busy: bool = False
    last_used: int = 0


class Scheduler:
    """Per-shape FIFO queues; lanes opened and released against an HBM budget.

    `executor` provides lane_plan(shape) -> (capacity, bytes), and
    create_lane(lane, shape, capacity) / destroy_lane(lane).  A lane id is
    (shape, k)."""

    def __init__(self, executor, budget_bytes, max_lanes_per_shape=4):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_lanes = max_lanes_per_shape
        self.queues = {}
        self.lanes = {}
        self.running = {}
        self.used = 0
        self.peak = 0
        self.waited_for_memory = set()   # ids of requests that had to wait for memory
        self.released = 0                # idle lanes released to make room
        self._tick = 0
        self._next = {}

    def arrive(self, req):
        _, nbytes = self.ex.lane_plan(req.shape)
        if nbytes > self.budget:
            raise ValueError("a lane of %s needs %.2f GB, more than the whole %.2f GB budget"
                             % (req.shape, nbytes / 1e9, self.budget / 1e9))
        self.queues.setdefault(req.shape, deque()).append(req)

    def _idle_lane(self, shape):
        best = None
        for lane, st in self.lanes.items():
            if st.shape == shape and not st.busy and (best is None or st.last_used > self.lanes[best].last_used):
                best = lane
        return best

    def _release_for(self, nbytes, keep_shape):
        """Release idle lanes of other shapes, least recently used first, until
        `nbytes` fit; True if they do."""
        idle = sorted((st.last_used, lane) for lane, st in self.lanes.items()
                      if not st.busy and st.shape != keep_shape)
        for _, lane in idle:
            if self.used + nbytes <= self.budget:
                break
            self.ex.destroy_lane(lane)
            self.used -= self.lanes.pop(lane).nbytes
            self.released += 1
        return self.used + nbytes <= self.budget

    def _open_lane(self, shape):
        """(new lane, None), or (None, "lanes") when the shape has its maximum
        of lanes, or (None, "memory") when the budget cannot take one more."""
        cap, nbytes = self.ex.lane_plan(shape)
        if sum(st.shape == shape for st in self.lanes.values()) >= self.max_lanes:
            return None, "lanes"
        if self.used + nbytes > self.budget and not self._release_for(nbytes, shape):
            return None, "memory"
        k = self._next.get(shape, 0)
        self._next[shape] = k + 1
        lane = (shape, k)
        self.ex.create_lane(lane, shape, cap)
        self.lanes[lane] = _LaneState(shape, cap, nbytes)
        self.used += nbytes
        self.peak = max(self.peak, self.used)
        return lane, None

    def dispatch(self):
        """[(lane, batch)] to launch now: shapes whose oldest request waited
        longest go first; each takes idle lanes of its shape, then new lanes
        while the budget allows.  Once a request waits for memory, younger
        shapes only reuse the lanes they have."""
        out = []
        blocked = False
        order = sorted((q[0].t_arrive, s) for s, q in self.queues.items() if q)
        for _, s in order:
            q = self.queues[s]
            while q:
                lane = self._idle_lane(s)
                if lane is None and not blocked:
                    lane, why = self._open_lane(s)
                    if why == "memory":
                        blocked = True
                        self.waited_for_memory.add(q[0].rid)
                if lane is None:
                    break
                st = self.lanes[lane]
                batch = [q.popleft() for _ in range(min(len(q), st.capacity))]
                st.busy = True
                self._tick += 1
                st.last_used = self._tick
                self.running[lane] = batch
                out.append((lane, batch))
        return out

    def complete(self, lane):
        batch = self.running.pop(lane)
        self.lanes[lane].busy = False
        return batch

    def busy_lanes(self):
        return list(self.running)

    def waiting(self):
        return sum(len(q) for q in self.queues.values())

    def idle(self):
        return not self.running and self.waiting() == 0

    def close(self):
        for lane in list(self.lanes):
            if not self.lanes[lane].busy:
                self.ex.destroy_lane(lane)
                self.used -= self.lanes.pop(lane).nbytes


def serve(requests, scheduler, executor, clock=time.perf_counter, sleep=time.sleep, progress=None):
    """Run the requests in real time (request i arrives t_arrive seconds after
    the start) and return them with t_start / t_done filled in.  `progress`,
    if given, is called about every 10 s of the run with (seconds, done)."""
    reqs = sorted(requests, key=lambda r: r.t_arrive)
    t0 = clock()
    i = done = 0
    next_note = 10.0
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
                done += len(batch)
                executor.finish(lane, batch)
                progressed = True
        for lane, batch in scheduler.dispatch():
            t = clock() - t0
            for r in batch:
                r.t_start = t
            executor.launch(lane, batch)
            progressed = True
        if progress and now >= next_note:
            progress(now, done)
            next_note += 10.0
        if not progressed:
            # poll while a lane runs or a request is due within a millisecond
            # (a timed sleep wakes up to ~0.3 ms late, which small pairs would
            # see in full); otherwise wake a little before the next arrival
            nxt = reqs[i].t_arrive - (clock() - t0) if i < len(reqs) else 0.0
            sleep(0.0 if scheduler.busy_lanes() or nxt < 1e-3 else nxt - 5e-4)
    return reqs


def summarize(reqs, duration=None):
    done = [r for r in reqs if not math.isnan(r.t_done)]
    lat = np.array([r.latency for r in done]) * 1e3
    span = duration if duration is not None else (max(r.t_done for r in done) - min(r.t_arrive for r in done))
    out = {"requests": len(reqs), "completed": len(done), "pairs_per_s": round(len(done) / span, 2) if span else None,
           "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
           "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
           "checked": sum(r.ok is not None for r in done), "mismatched": sum(r.ok is False for r in done)}
    dev = np.array([r.device_ms for r in done if not math.isnan(r.device_ms)])
    if len(dev):
        out["device_p50_ms"] = round(float(np.percentile(dev, 50)), 3)
        out["device_p99_ms"] = round(float(np.percentile(dev, 99)), 3)
    per = {}
    for s in sorted({r.shape for r in done}):
        ls = np.array([r.latency for r in done if r.shape == s]) * 1e3
        per[s] = {"n": int(len(ls)), "p50_ms": round(float(np.percentile(ls, 50)), 3),
                  "p99_ms": round(float(np.percentile(ls, 99)), 3)}
        ds = np.array([r.device_ms for r in done if r.shape == s and not math.isnan(r.device_ms)])
        if len(ds):
            per[s]["device_p50_ms"] = round(float(np.percentile(ds, 50)), 3)
            per[s]["device_p99_ms"] = round(float(np.percentile(ds, 99)), 3)
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
    event: object           # completion of the last launch (after the download)
    solve0: object          # timing events around the batch's kernels
    solve1: object
    graphs: dict = field(default_factory=dict)


class GpuExecutor:
    """Lanes on the device, opened and released by the scheduler.

    pairs: {shape name: [StereoPair, ...]} -- the inputs requests refer to;
      shape names are "<W>x<H>_d<D>", any size and disparity range.
    lane_bytes: the size a lane aims at; its batch capacity is that over one
      pair's bytes, between 1 and max_batch.
    graphs: replay library-captured graphs (else eager stereo_solve_batch).
    check: compare every result with the pair solved alone (bit for bit)."""

    def __init__(self, pairs, vol_dtype=None, budget_bytes=64 * 10 ** 9, lane_bytes=1 << 30, max_batch=8,
                 max_lanes_per_shape=4, radius=4, sigma_s=20.0, sigma_r=0.1, dt_iters=3, graphs=True, check=True,
                 autotune_cache=None, device="cuda"):
        import torch

        from . import _lib as lib
        self.torch, self.lib = torch, lib
        self.vol_dtype = lib.ZDT_F16 if vol_dtype is None else vol_dtype
        self.budget, self.lane_target, self.max_batch = budget_bytes, lane_bytes, max_batch
        self.max_lanes = max_lanes_per_shape
        self.pp = (radius, sigma_s, sigma_r, dt_iters)
        self.use_graphs, self.check, self.autotune_cache = graphs, check, autotune_cache
        self.dev = torch.device(device)
        self.params, self.lanes, self.alone = {}, {}, {}
        self.graph_captures = 0
        self.pinned = {s: [(torch.from_numpy(p.left).pin_memory(), torch.from_numpy(p.right).pin_memory())
                           for p in ps] for s, ps in pairs.items()}
        if check:
            for s in self.pinned:
                self.alone[s] = [self._solve_alone(s, i) for i in range(len(self.pinned[s]))]

    # -- shapes
    def _params(self, s):
        if s not in self.params:
            sh = shape_of(s)
            p = self.lib.params(sh.W, sh.H, sh.D, *self.pp, vol_dtype=self.vol_dtype)
            if self.autotune_cache:
                self.lib.autotune(p, self.autotune_cache)
            self.params[s] = p
        return self.params[s]

    def pair_bytes(self, s):
        sh, p = shape_of(s), self._params(s)
        return self.lib.volume_size(p) + self.lib.workspace_size(p) + sh.W * sh.H * (2 + 4)

    def lane_plan(self, s):
        per = self.pair_bytes(s)
        cap = max(1, min(self.max_batch, self.lane_target // per))
        return cap, cap * per

    def scheduler(self):
        return Scheduler(self, self.budget, self.max_lanes)

    # -- lanes
    def create_lane(self, lane_id, s, cap):
        torch, lib = self.torch, self.lib
        sh, p = shape_of(s), self._params(s)
        wsz = lib.workspace_size(p)
        u8 = dict(dtype=torch.uint8, device=self.dev)
        left, right = torch.empty((cap, sh.H, sh.W), **u8), torch.empty((cap, sh.H, sh.W), **u8)
        disp = torch.empty((cap, sh.H, sh.W), dtype=torch.int32, device=self.dev)
        vols = [torch.empty(lib.volume_size(p), **u8) for _ in range(cap)]
        wss = [torch.empty(wsz, **u8) if wsz else None for _ in range(cap)]
        jobs = [(p, left[i], right[i], disp[i], vols[i], wss[i]) for i in range(cap)]
        host_out = torch.empty((cap, sh.H, sh.W), dtype=torch.int32).pin_memory()
        self.lanes[lane_id] = _Lane(sh, torch.cuda.Stream(device=self.dev), left, right, disp, host_out, vols, wss,
                                    jobs, torch.cuda.Event(), torch.cuda.Event(enable_timing=True),
                                    torch.cuda.Event(enable_timing=True))

    def destroy_lane(self, lane_id):
        lane = self.lanes.pop(lane_id)
        lane.stream.synchronize()
        for g in lane.graphs.values():
            g.close()

    def _solve_alone(self, s, i):
        torch, lib = self.torch, self.lib
        sh, p = shape_of(s), self._params(s)
        left, right = (t.to(self.dev) for t in self.pinned[s][i])
        disp = torch.empty((sh.H, sh.W), dtype=torch.int32, device=self.dev)
        vol = torch.empty(lib.volume_size(p), dtype=torch.uint8, device=self.dev)
        wsz = lib.workspace_size(p)
        ws = torch.empty(wsz, dtype=torch.uint8, device=self.dev) if wsz else None
        lib.stereo_solve(p, left, right, disp, vol, ws)
        out = disp.cpu().numpy()
        del vol, ws
        return out

    def launch(self, lane_id, batch):
        torch, lane = self.torch, self.lanes[lane_id]
        n = len(batch)
        with torch.cuda.stream(lane.stream):
            for k, r in enumerate(batch):
                src_l, src_r = self.pinned[r.shape][r.pair]
                lane.left[k].copy_(src_l, non_blocking=True)
                lane.right[k].copy_(src_r, non_blocking=True)
            lane.solve0.record(lane.stream)
            if not self.use_graphs:
                self.lib.stereo_solve_batch(lane.jobs[:n], stream=lane.stream)
            elif n in lane.graphs:
                lane.graphs[n].launch(lane.stream)
            else:   # capturing runs the batch once, eagerly, before recording it
                lane.graphs[n] = self.lib.Graph(lane.jobs[:n], lane.stream)
                self.graph_captures += 1
            lane.solve1.record(lane.stream)
            lane.host_out[:n].copy_(lane.disp[:n], non_blocking=True)
            lane.event.record(lane.stream)

    def poll(self, lane_id):
        return self.lanes[lane_id].event.query()

    def finish(self, lane_id, batch):
        lane = self.lanes[lane_id]
        dev_ms = lane.solve0.elapsed_time(lane.solve1)
        for r in batch:
            r.device_ms = dev_ms
        if not self.check:
            return
        for k, r in enumerate(batch):
            r.ok = bool(np.array_equal(lane.host_out[k].numpy(), self.alone[r.shape][r.pair]))


def per_pair_capacity(reqs, pairs, vol_dtype, radius=4, sigma_s=20.0, sigma_r=0.1, dt_iters=3):
    """Pairs per second of the plain form: the same requests solved one at a
    time on one stream (upload, stereo_solve, download), no batching, no graphs."""
    import torch

    from . import _lib as lib
    bufs = {}
    for name in {r.shape for r in reqs}:
        sh = shape_of(name)
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


def _one_pair(args):
    from . import scenes
    w, h, d, seed = args
    return scenes.planes_pair(w, h, d, seed=seed)


def make_pairs(per_shape, shapes=SHAPES, seed=1000, workers=1):
    """Input pools: `per_shape[name]` synthetic scenes of each shape (seeds
    seed + 17 i + W), generated on `workers` processes."""
    jobs = [(s.name, (s.W, s.H, s.D, seed + 17 * i + s.W)) for s in shapes for i in range(per_shape.get(s.name, 0))]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            made = list(ex.map(_one_pair, [a for _, a in jobs]))
    else:
        made = [_one_pair(a) for _, a in jobs]
    out = {}
    for (name, _), pr in zip(jobs, made):
        out.setdefault(name, []).append(pr)
    return out


def run(rate=300.0, duration=60.0, vol_dtype=None, pairs_per_shape=64, graphs=True, check=True, seed=7, workers=16,
        progress=None):
    """Serve a Poisson stream of the mixed shapes (pools of `pairs_per_shape`
    seeded pairs each, generated before the clock starts) and summarise it."""
    pools = make_pairs({s.name: pairs_per_shape for s in SHAPES}, workers=workers)
    ex = GpuExecutor(pools, vol_dtype=vol_dtype, graphs=graphs, check=check)
    sched = ex.scheduler()
    reqs = poisson_arrivals(rate, duration, MIX, {k: len(v) for k, v in pools.items()}, seed=seed)
    serve(reqs, sched, ex, progress=progress)
    out = summarize(reqs, duration=duration)
    out.update({"offered_per_s": rate, "seconds": duration, "pairs_per_shape": pairs_per_shape,
                "budget_gb": round(ex.budget / 1e9, 2), "peak_lane_bytes_gb": round(sched.peak / 1e9, 3),
                "lanes_opened": {s: n for s, n in sched._next.items()}, "graph_captures": ex.graph_captures,
                "waited_for_memory": len(sched.waited_for_memory), "lanes_released": sched.released,
                "graphs": graphs})
    sched.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--rate", type=float, default=300.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    print(json.dumps(run(args.rate, args.duration, pairs_per_shape=args.pairs, graphs=not args.no_graphs,
                         check=not args.no_check)))


if __name__ == "__main__":
    main()
