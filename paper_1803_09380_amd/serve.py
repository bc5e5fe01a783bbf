"""Continuous batching of simulation requests on one GPU.

Requests (a case from workloads.py, a step budget and an arrival time) are
admitted into one running batch whenever the batch's HBM budget allows; their
state stays on the device; the batch advances all admitted requests together
in chunks of steps; a request whose budget is spent stops by itself on the
device (its step counter reaches zero inside the batch) and is retired,
read out and freed between chunks, which makes room for waiting requests.

The policy (admission order, budget, chunking, completion) is written against
a small executor interface so it can be tested on the CPU with a mock; the
GPU executor maps it onto the batch calls of the C ABI, and all the
simulation work runs in the library's kernels.
"""
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrive: float
    case: dict
    steps: int
    t_admit: float = None
    t_done: float = None
    result: dict = None


class GpuExecutor:
    """Executor over lbmib.Batch (one precision, one HBM budget)."""

    def __init__(self, precision, hbm_budget, tiling=None, lanes=None, halves_from=5):
        """lanes: the batch's lane mode (lbmib.Batch.set_lanes), None for the
        library's choice.  halves_from > 0: two interleaved halves (lane mode
        4, one half's correction beside the other half's sweep) while at
        least that many requests are on the device, set afresh at every
        admission and retirement; the library's choice below that (one lane
        costs less with few members).  0: never."""
        from . import lbmib
        self.lbmib = lbmib
        self.batch = lbmib.Batch(precision, hbm_budget=hbm_budget)
        self.precision = precision
        if tiling is not None:
            self.batch.set_tiling(tiling)
        if lanes is not None:
            self.batch.set_lanes(lanes)
        self.halves_from = halves_from
        self.halves = False
        self.live = {}

    def _lanes(self):
        want = self.halves_from > 0 and len(self.live) >= self.halves_from
        if want or self.halves:
            self.batch.set_lanes(4 if want else 0)
        self.halves = want

    def create(self, req):
        return self.lbmib.Sim.from_case(req.case, precision=self.precision)

    def bytes_needed(self, req):
        """Device memory a request will hold, bounded on the host before
        anything is created."""
        return self.lbmib.device_bytes_bound(req.case, self.precision)

    def bytes(self, handle):
        return handle.device_bytes

    def admit(self, req, handle):
        ok = self.batch.admit(handle, steps=req.steps)
        if ok:
            self.live[req.rid] = handle
            self._lanes()
        return ok

    def step(self, n):
        self.batch.step(n)

    def sync(self):
        import torch
        torch.cuda.synchronize()

    def finish(self, req):
        h = self.live.pop(req.rid)
        self.batch.retire(h)
        self._lanes()
        res = {"steps": h.step_count, "bodies": [h.forces(k) for k in range(len(req.case["bodies"]))]}
        h.close()
        return res

    def discard(self, handle):
        handle.close()

    def close(self):
        self.batch.close()


@dataclass
class Stats:
    latencies: list = field(default_factory=list)
    updates: int = 0
    wall: float = 0.0
    max_live: int = 0
    queue_peak: int = 0
    timeline: list = field(default_factory=list)  # (time, requests on the device, requests queued) per chunk

    def summary(self, points=32):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        tl = self.timeline
        if len(tl) > points:
            tl = [tl[int(round(k * (len(tl) - 1) / (points - 1)))] for k in range(points)]
        return {"requests": len(self.latencies), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                "aggregate_mlups": self.updates / self.wall / 1e6 if self.wall > 0 else 0.0,
                "max_concurrent": self.max_live, "queue_peak": self.queue_peak, "wall_s": self.wall,
                "timeline_s_live_queued": [[round(t, 3), a, q] for t, a, q in tl]}


class Server:
    """Continuous-batching loop.  `clock` returns seconds since the start and
    `sleep` waits (wall clock by default; the mock tests pass virtual ones)."""

    def __init__(self, executor, hbm_budget, chunk=50, clock=None, sleep=None):
        self.ex = executor
        self.budget = hbm_budget
        self.chunk = chunk
        t0 = time.perf_counter()
        self.clock = clock or (lambda: time.perf_counter() - t0)
        self.sleep = sleep or time.sleep
        self.used = 0
        self.live = []  # (req, handle, bytes, steps enqueued since admission)
        self.stats = Stats()

    def _try_admit(self, waiting):
        """Admit waiting requests in arrival order while the budget allows;
        stops at the first one that does not fit (no overtaking).  The fit is
        decided on the executor's host-side bound of the request's memory, so
        a request that has to wait costs no device allocation; once admitted
        it is charged what it actually holds."""
        while waiting:
            req = waiting[0]
            need = self.ex.bytes_needed(req)
            if self.budget and self.used + need > self.budget:
                if not self.live and need > self.budget:
                    raise ValueError("request %d needs %d bytes, above the whole budget" % (req.rid, need))
                return
            handle = self.ex.create(req)
            nb = self.ex.bytes(handle)
            if not self.ex.admit(req, handle):
                self.ex.discard(handle)
                return
            waiting.pop(0)
            req.t_admit = self.clock()
            self.used += nb
            self.live.append([req, handle, nb, 0])
            self.stats.max_live = max(self.stats.max_live, len(self.live))

    def run(self, requests):
        pending = sorted(requests, key=lambda r: r.t_arrive)
        waiting = []
        done = []
        start = self.clock()
        while pending or waiting or self.live:
            now = self.clock()
            while pending and pending[0].t_arrive <= now:
                waiting.append(pending.pop(0))
            self.stats.queue_peak = max(self.stats.queue_peak, len(waiting))
            self._try_admit(waiting)
            if not self.live:
                if pending:
                    self.sleep(max(0.0, pending[0].t_arrive - self.clock()))
                continue
            # advance the batch by one chunk (members stop on their own budgets)
            self.stats.timeline.append((now - start, len(self.live), len(waiting)))
            n = min(self.chunk, max(r[0].steps - r[3] for r in self.live))
            self.ex.step(n)
            self.ex.sync()
            now = self.clock()
            keep = []
            for entry in self.live:
                req, handle, nb, enq = entry
                ran = min(n, req.steps - enq)
                entry[3] = enq + n
                self.stats.updates += req.case["nx"] * req.case["ny"] * ran
                if entry[3] >= req.steps:
                    req.result = self.ex.finish(req)
                    req.t_done = now
                    self.used -= nb
                    self.stats.latencies.append(req.t_done - req.t_arrive)
                    done.append(req)
                else:
                    keep.append(entry)
            self.live = keep
        self.stats.wall = self.clock() - start
        return done
