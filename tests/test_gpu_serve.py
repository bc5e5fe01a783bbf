"""Serving on the GPU: requests that arrive while others run are admitted into
the running batch as the HBM budget frees up, and each result is bitwise the
same as the request run alone."""
import sys

import numpy as np
import pytest

from gpu_helpers import gpu_from_case
from paper_1803_09380_amd import lbmib
from paper_1803_09380_amd import workloads as wl
from paper_1803_09380_amd.serve import GpuExecutor, Request, Server

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    print("serve 6 requests", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(7)
    reqs = []
    for k in range(6):
        case = wl.settling(nx=60, ny=200, D=float(rng.uniform(10, 14)), density_ratio=float(rng.uniform(1.1, 1.5)),
                           two=bool(k % 2), lower=(30.0, 120.0), u_ref=0.05)
        reqs.append(Request(rid=k, t_arrive=0.002 * k, case=case, steps=int(60 + 20 * k)))
    one = gpu_from_case(reqs[0].case, precision=lbmib.F32_SHIFTED)
    budget = int(one.device_bytes * 3.5)
    one.close()
    ex = GpuExecutor(lbmib.F32_SHIFTED, hbm_budget=budget)
    srv = Server(ex, hbm_budget=budget, chunk=25)
    done = srv.run(reqs)
    ex.close()
    assert len(done) == 6
    assert srv.stats.max_live <= 3
    for r in done:
        alone = gpu_from_case(r.case, precision=lbmib.F32_SHIFTED)
        alone.step(r.steps)
        assert r.result["steps"] == r.steps
        for k, got in enumerate(r.result["bodies"]):
            ref = alone.forces(k)
            assert np.array_equal(got[0], ref[0]) and got[1] == ref[1]
            assert np.array_equal(got[3], ref[3])
    s = srv.stats.summary()
    assert s["p99_s"] >= s["p50_s"] > 0
