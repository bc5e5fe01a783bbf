"""CPU tests of the continuous-batching policy with a mock executor on a
virtual clock (no GPU): admission by HBM budget in arrival order, overlap of
requests, completion at the step budget, latency accounting."""
import numpy as np
import pytest

from paper_1803_09380_amd import workloads as wl
from paper_1803_09380_amd.serve import Request, Server


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-9)


class MockExecutor:
    """Costs one virtual second per 1e8 node updates of the whole batch."""

    def __init__(self, clock, bytes_per_node=36):
        self.clock = clock
        self.bpn = bytes_per_node
        self.live = {}
        self.trace = []

    def create(self, req):
        self.trace.append(("create", req.rid, self.clock()))
        return {"rid": req.rid, "nodes": req.case["nx"] * req.case["ny"], "left": req.steps, "ran": 0}

    def bytes_needed(self, req):
        return req.case["nx"] * req.case["ny"] * self.bpn

    def bytes(self, h):
        return h["nodes"] * self.bpn

    def admit(self, req, h):
        self.live[req.rid] = h
        self.trace.append(("admit", req.rid, self.clock()))
        return True

    def step(self, n):
        work = 0
        for h in self.live.values():
            k = min(n, h["left"])
            h["left"] -= k
            h["ran"] += k
            work += k * h["nodes"]
        self.clock.t += work / 1e8

    def sync(self):
        pass

    def finish(self, req):
        h = self.live.pop(req.rid)
        self.trace.append(("done", req.rid, self.clock()))
        return {"steps": h["ran"]}

    def discard(self, h):
        pass


def _reqs(n, rate, steps, nx=100, ny=400, seed=1):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return [Request(rid=k, t_arrive=float(t[k]),
                    case=wl.settling(nx=nx, ny=ny, D=12.0, density_ratio=1.2, lower=(nx / 2, ny - 50.0)),
                    steps=steps) for k in range(n)]


def test_every_request_runs_exactly_its_budget():
    clk = VirtualClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=0, chunk=37, clock=clk, sleep=clk.sleep)
    reqs = _reqs(12, rate=50.0, steps=300)
    done = srv.run(reqs)
    assert len(done) == 12
    assert all(r.result["steps"] == 300 for r in done)
    s = srv.stats.summary()
    assert s["requests"] == 12 and s["p99_s"] >= s["p50_s"] > 0
    assert srv.stats.updates == 12 * 300 * 100 * 400


def test_budget_limits_concurrency_and_keeps_arrival_order():
    clk = VirtualClock()
    ex = MockExecutor(clk)
    per = 100 * 400 * 36
    srv = Server(ex, hbm_budget=3 * per, chunk=50, clock=clk, sleep=clk.sleep)
    reqs = _reqs(10, rate=1000.0, steps=200)  # all arrive almost at once
    done = srv.run(reqs)
    assert len(done) == 10
    assert srv.stats.max_live == 3
    admits = [rid for kind, rid, _ in ex.trace if kind == "admit"]
    assert admits == sorted(admits)
    assert srv.stats.queue_peak >= 5
    # the timeline of requests on the device and queued: never more than the
    # budget allows, queued requests drain, times increase
    tl = srv.stats.summary(points=8)["timeline_s_live_queued"]
    assert 2 <= len(tl) <= 8
    assert all(0 < a <= 3 for _, a, _ in tl) and max(q for _, _, q in tl) >= 5 and tl[-1][2] == 0
    assert all(t1 >= t0 for (t0, _, _), (t1, _, _) in zip(tl, tl[1:]))


def test_requests_arriving_while_others_run_are_admitted_between_chunks():
    clk = VirtualClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=0, chunk=20, clock=clk, sleep=clk.sleep)
    r0 = Request(0, 0.0, wl.settling(nx=100, ny=400, D=12.0, lower=(50.0, 350.0)), 400)
    r1 = Request(1, 0.05, wl.settling(nx=100, ny=400, D=12.0, lower=(50.0, 350.0)), 100)
    done = srv.run([r0, r1])
    t = {(k, rid): tt for k, rid, tt in ex.trace}
    # r1 joined before r0 finished and finished first
    assert t[("admit", 1)] < t[("done", 0)]
    assert t[("done", 1)] < t[("done", 0)]
    assert {r.rid for r in done} == {0, 1}


def test_request_larger_than_the_budget_is_refused():
    clk = VirtualClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=1000, chunk=20, clock=clk, sleep=clk.sleep)
    with pytest.raises(ValueError):
        srv.run(_reqs(1, rate=10.0, steps=10))


def test_idle_server_waits_for_the_next_arrival():
    clk = VirtualClock()
    ex = MockExecutor(clk)
    srv = Server(ex, hbm_budget=0, chunk=50, clock=clk, sleep=clk.sleep)
    reqs = [Request(0, 5.0, wl.settling(nx=100, ny=400, D=12.0, lower=(50.0, 350.0)), 50)]
    done = srv.run(reqs)
    assert done[0].t_admit >= 5.0


def test_no_request_is_created_while_admission_is_blocked():
    """A request that does not fit the budget waits without a device
    allocation: each request is created once, when it is admitted."""
    clk = VirtualClock()
    ex = MockExecutor(clk)
    per = 100 * 400 * 36
    srv = Server(ex, hbm_budget=2 * per, chunk=25, clock=clk, sleep=clk.sleep)
    done = srv.run(_reqs(8, rate=1000.0, steps=150))
    assert len(done) == 8
    creates = [rid for kind, rid, _ in ex.trace if kind == "create"]
    admits = [rid for kind, rid, _ in ex.trace if kind == "admit"]
    assert creates == admits == list(range(8))
    # every create is immediately followed by its admit
    kinds = [(kind, rid) for kind, rid, _ in ex.trace if kind in ("create", "admit")]
    assert all(kinds[2 * k] == ("create", k) and kinds[2 * k + 1] == ("admit", k) for k in range(8))
