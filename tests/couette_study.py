"""Convergence study of the cylindrical Couette flow of Sec. 3.1.2.

The paper's own set-up (workloads.couette_paper): MRT with the rates of
Sec. 4.1, Re = 10, tau_s = 0.65 and 0.85, radius ratio R = 0.5 and 0.8, outer
radius resolved by N = 20, 40, 80 lattice spacings, run to steady state.
Refinement keeps tau_s and Re, so the lattice wall speed falls as 1/N: an
error measured in lattice velocity units gains one order from that alone.
The scale-free measure is the error relative to the wall speed U1 = omega1 R1,
which is also the error in physical units at a fixed physical wall speed.

Reported per run, against Eq. 34: the Eq. 35 norm on the theta = pi/2
profile in lattice units and relative to U1, and the relative error over all
annulus nodes; per parameter set, the least-squares orders of each.

    python tests/couette_study.py [--grids 20 40 80] [--jobs 4] [--write-golden]

runs the study on the FP64 CPU oracle (test infrastructure; minutes);
--write-golden stores the oracle's errors in tests/golden/couette_paper_oracle.json,
which the GPU test of the same set-up compares against.
"""
import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, os.path.join(ROOT, "oracle")):
    if p not in sys.path:
        sys.path.insert(0, p)

from paper_1803_09380_amd import diagnostics as dg  # noqa: E402
from paper_1803_09380_amd import workloads as wl  # noqa: E402

SETS = [(0.5, 0.65), (0.5, 0.85), (0.8, 0.65), (0.8, 0.85)]  # (radius ratio R, tau_s)


def errors(case, ux, uy):
    """(Eq. 35 norm in lattice units, the same relative to U1, relative error
    over the annulus nodes) of a steady field."""
    m = case["meta"]
    rel, e35 = dg.couette_errors(ux, uy, m["centre"], m["R1"], m["R2"], m["omega1"])
    return e35, e35 / m["U1"], rel


def run_oracle(N, ratio, tau):
    import pyoracle as po
    case = wl.couette_paper(N, ratio, tau)
    o = po.Oracle(case["nx"], case["ny"], case["tau"], bc=case["bc"], collision=po.MRT,
                  mrt_s=case["mrt_s"], ib_iters=case["ib_iters"])
    for k, b in enumerate(case["bodies"]):
        o.set_body(k, b["kind"], b["n"], xy=b["xy"], ds=b["ds"], xc=b["xc"], omega=b["omega"])
    o.step(case["meta"]["steps"])
    _, ux, uy = o.fields()
    return errors(case, ux, uy)


def orders(grids, rows):
    """Least-squares orders (positive = error falls with N) of each column."""
    h = 1.0 / np.asarray(grids, dtype=np.float64)
    cols = list(zip(*rows))
    return [dg.observed_order(h, c) for c in cols]


def _job(args):
    N, ratio, tau = args
    return (N, ratio, tau), run_oracle(N, ratio, tau)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--grids", type=int, nargs="+", default=[20, 40, 80])
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--write-golden", action="store_true")
    args = ap.parse_args()
    import multiprocessing as mp
    os.environ.setdefault("OMP_NUM_THREADS", str(max(1, (os.cpu_count() or 1) // args.jobs)))
    work = [(N, r, t) for (r, t) in SETS for N in args.grids]
    with mp.Pool(args.jobs) as pool:
        res = dict(pool.map(_job, work))
    out = []
    for r, t in SETS:
        rows = [res[(N, r, t)] for N in args.grids]
        o = orders(args.grids, rows)
        out.append({"R": r, "tau_s": t, "grids": args.grids,
                    "eq35_lattice": [x[0] for x in rows], "eq35_relative": [x[1] for x in rows],
                    "annulus_relative": [x[2] for x in rows],
                    "order_eq35_lattice": o[0], "order_eq35_relative": o[1], "order_annulus_relative": o[2]})
        print(json.dumps(out[-1]), flush=True)
    if args.write_golden:
        path = os.path.join(HERE, "golden", "couette_paper_oracle.json")
        with open(path, "w") as f:
            json.dump({"source": "tests/couette_study.py on the FP64 CPU oracle (oracle/lbm_oracle.c); "
                                 "cylindrical Couette flow as set up in Sec. 3.1.2 (workloads.couette_paper), "
                                 "errors against Eq. 34",
                       "columns": ["eq35_lattice", "eq35_relative", "annulus_relative"], "sets": out}, f, indent=1)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
