#!/usr/bin/env python3
"""Benchmark of the MI355X IB-LBM hot path.

Workload: the batched uneven set -- 256 seeded simulations, each either a
cylindrical Couette case (side uniform in 64..512) or a fixed cylinder in a
20D x 10D channel (D uniform in 16..64, Re uniform in 10..100), FP32 shifted
populations, all advanced together by the batch (captured graphs of persistent
kernels).  One step = collide-stream sweep, boundary rules, 10 correction
sweeps with FP64 force/torque reductions, bookkeeping, for every member.

Printed (one JSON line): aggregate MLUPS of the batched FP32 path over exactly
--steps timed steps; the sweep kernel's HBM roofline fraction (per-launch
duration from HIP events on the batch stream) against the datasheet peak and
against the best copy measured here (copy_probe.py), and the whole step's
fraction at 72 B per node update; the plain per-simulation FP64 GPU path on a
sample of the same set; the set with the MRT collision; the served stream
(arrival-bound and overloaded); and the FP64 CPU oracle timed on the host
cores (one thread and every thread, CPU model stated) on a bounded sample,
with every GPU path's error against it on seeded members of the same
workloads.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D2Q9+IB MLUPS (FP32 batched vs FP64 plain) at stated error; p50/p99 solve time"
HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_F32 = 72  # 9 loads + 9 stores of 4 bytes per cell update
SWEEP_BYTES_F64 = 144
# HBM counter figures of the sweep on this set, per tiling, from two
# `rocprofv3 --pmc` passes (FETCH_SIZE, WRITE_SIZE) scaled by the same
# counters' reading for a plain copy of known size; they hold only for the
# kernel source they were taken on (its SHA-256 is recorded with them).
PMC_FILE = os.path.join(ROOT, "profiles", "k_sweep_f32_batched256_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1803_09380_amd", "csrc", "kernels.hip")


def frac_of_peak(mlups):
    """Fraction of the HBM peak that `mlups` FP32 node updates per second
    would move at the sweep's 72 algorithmic bytes each."""
    return None if mlups is None else round(mlups * SWEEP_BYTES_F32 / 1e3 / HBM_PEAK_GBS, 4)


def sweep_traffic(tiling):
    """HBM bytes per sweep launch for `tiling` from the committed counter
    summary, or None when there is none for this tiling or the kernel source
    has changed since the counters were taken."""
    import hashlib
    try:
        lines = open(PMC_FILE).read().splitlines()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    rec, rows = {}, {}
    for ln in lines:
        f = ln.split()
        if not f or f[0].startswith("#") or f[0].startswith("|"):
            continue
        if f[0] == "tiling" and len(f) >= 6:
            rows[int(f[1])] = (float(f[3]), float(f[5]))
        elif len(f) == 2:
            rec[f[0]] = f[1]
    if rec.get("kernel_source_sha256") != sha or tiling not in rows:
        return None
    fk, wk = rows[tiling]
    return (fk * float(rec["fetch_factor"]) + wk * float(rec["write_factor"])) * 1024.0


def _oracle_from_case(po, case):
    o = po.Oracle(case["nx"], case["ny"], case["tau"], rho0=case["rho0"], bc=case["bc"], u_in=case["u_in"],
                  u_init=case["u_init"], ib_iters=case["ib_iters"], gravity=case["gravity"])
    for k, b in enumerate(case["bodies"]):
        if b["kind"] == 1:
            o.set_body(k, po.FREE, b["n"], xc=b["xc"], U=b["U"], omega=b["omega"], theta=b["theta"],
                       radius=b["radius"], rho_s=b["rho_s"])
        else:
            o.set_body(k, po.FIXED, b["n"], xy=b["xy"], uv=b["uv"], ds=b["ds"], xc=b["xc"], U=b["U"],
                       omega=b["omega"], theta=b["theta"])
    return o


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _host_threads():
    """Threads the oracle may use: the host cores this process may run on,
    at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_sample(po, cases, seconds, max_steps=200):
    """Time the oracle on members of `cases` one at a time, in seed order,
    until `seconds` of host time are used (each member at least 5 steps)."""
    updates, used, steps_each = 0, 0.0, []
    for case in cases:
        if used >= seconds:
            break
        o = _oracle_from_case(po, case)
        n, t0 = 0, time.perf_counter()
        while True:
            o.step(5)
            n += 5
            el = time.perf_counter() - t0
            if el > seconds / 4 or used + el >= seconds or n >= max_steps:
                break
        used += el
        updates += case["nx"] * case["ny"] * n
        steps_each.append(n)
    return {"updates": updates, "seconds": used, "members": len(steps_each), "steps": steps_each}


def _cpu_configs():
    """Seeded cases of the other configurations, each timed on a bounded
    number of steps: (name, case, steps)."""
    from paper_1803_09380_amd import workloads as wl
    out = [("couette64", wl.couette(64), 2000), ("couette256", wl.couette(256), 100),
           ("cylinder1600x800_re20", wl.cylinder(Re=20.0), 2000)]
    for k, r in enumerate(wl.arrivals(seed=0, rate=20.0, count=4, steps=2000)):
        out.append(("served_request%d" % k, r["case"], 10))
    return out


def cpu_worker(spec):
    """Child process of the CPU baseline: OMP_NUM_THREADS is fixed by the
    parent.  Prints one JSON line."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle as po
    po.build()
    from paper_1803_09380_amd import workloads as wl
    if spec["kind"] == "batch":
        cases = wl.batch(seed=spec["seed"], count=spec["sims"], precision=wl.F32)
        res = _oracle_sample(po, cases[:16], spec["seconds"])
    else:
        res = {}
        for name, case, steps in _cpu_configs():
            print("cpu baseline: %s, %d steps, %s threads" % (name, steps, os.environ.get("OMP_NUM_THREADS")),
                  file=sys.stderr, flush=True)
            o = _oracle_from_case(po, case)
            o.step(1)
            t0 = time.perf_counter()
            o.step(steps)
            el = time.perf_counter() - t0
            res[name] = {"mlups": round(case["nx"] * case["ny"] * steps / el / 1e6, 3), "steps": steps,
                         "nodes": case["nx"] * case["ny"], "seconds": round(el, 3)}
    print(json.dumps(res), flush=True)


def _run_worker(spec, threads):
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OMP_PROC_BIND="false")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker", json.dumps(spec)],
                         stdout=subprocess.PIPE, text=True, env=env, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def run_cpu_baseline(args):
    """The FP64 oracle on the host cores: the first members of the set one at
    a time, single-threaded and with every thread this process may use (in
    child processes, before the GPU is touched); optionally the other
    configurations on bounded step counts."""
    threads = _host_threads()
    spec = {"kind": "batch", "seed": args.seed, "sims": args.sims, "seconds": args.cpu_seconds / 2}
    one = _run_worker(spec, 1)
    alln = _run_worker(spec, threads) if threads > 1 else one
    res = {"value": round(alln["updates"] / alln["seconds"] / 1e6, 3), "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": "first %d members of the set one at a time, %s steps each, %.1f s of host time "
                     "(FP64; collide/stream OpenMP over %d threads, correction serial)"
                     % (alln["members"], alln["steps"], alln["seconds"], threads),
           "single_thread": {"value": round(one["updates"] / one["seconds"] / 1e6, 3), "unit": "MLUPS",
                             "sample": "first %d members, %s steps each, %.1f s"
                                       % (one["members"], one["steps"], one["seconds"])},
           "cpu_model": _cpu_model()}
    if args.cpu_configs:
        res["configs"] = {"threads_1": _run_worker({"kind": "configs"}, 1)}
        if threads > 1:
            res["configs"]["threads_%d" % threads] = _run_worker({"kind": "configs"}, threads)
    return res


def _vel_err(g, o):
    import numpy as np
    _, ug, vg = g
    _, uo, vo = o
    l2 = float(np.sqrt(np.sum((ug - uo) ** 2 + (vg - vo) ** 2) / np.sum(uo ** 2 + vo ** 2)))
    mx = float(max(np.abs(ug - uo).max(), np.abs(vg - vo).max()) / max(np.abs(uo).max(), np.abs(vo).max()))
    return {"velocity_rel_l2": l2, "velocity_max_rel": mx}


def oracle_errors(cases, lbmib, wl, steps=100):
    """Part of the CPU-baseline leg: each GPU path against the FP64 oracle on
    the same seeded input -- the smallest Couette and the smallest cylinder of
    the set (FP32 shifted as batched, and FP64 as the plain path), the
    smallest Couette with the MRT rates, and one served request (a 400 x 4000
    box, 10 steps).  A member gives the same bits alone and in the batch, so
    it runs alone here."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle as po
    po.build()
    cou = min((c for c in cases if c["bodies"] and c["bc"][0] == wl.PERIODIC), key=lambda c: c["nx"] * c["ny"])
    cyl = min((c for c in cases if c["bc"][0] != wl.PERIODIC), key=lambda c: c["nx"] * c["ny"])
    out = {"steps": steps}
    for name, case in (("couette_%dx%d" % (cou["nx"], cou["ny"]), cou),
                       ("cylinder_%dx%d" % (cyl["nx"], cyl["ny"]), cyl)):
        o = _oracle_from_case(po, case)
        o.step(steps)
        of = o.fields()
        row = {}
        for pname, prec in (("fp32_shifted", lbmib.F32_SHIFTED), ("fp64", lbmib.F64)):
            g = lbmib.Sim.from_case(case, precision=prec)
            g.step(steps)
            row[pname] = _vel_err(g.fields(), of)
            g.close()
        out[name] = row
    rates = wl.mrt_rates(cou["tau"])
    o = po.Oracle(cou["nx"], cou["ny"], cou["tau"], rho0=cou["rho0"], bc=cou["bc"], u_in=cou["u_in"],
                  u_init=cou["u_init"], ib_iters=cou["ib_iters"], gravity=cou["gravity"], collision=po.MRT,
                  mrt_s=rates)
    for k, b in enumerate(cou["bodies"]):
        o.set_body(k, po.FIXED, b["n"], xy=b["xy"], uv=b["uv"], ds=b["ds"], xc=b["xc"], U=b["U"],
                   omega=b["omega"], theta=b["theta"])
    o.step(steps)
    g = lbmib.Sim.from_case(cou, precision=lbmib.F32_SHIFTED, mrt_s=rates)
    g.step(steps)
    out["mrt_fp32_shifted"] = _vel_err(g.fields(), o.fields())
    g.close()
    req = wl.arrivals(seed=0, rate=20.0, count=1, steps=2000)[0]["case"]
    o = _oracle_from_case(po, req)
    o.step(10)
    g = lbmib.Sim.from_case(req, precision=lbmib.F32_SHIFTED)
    g.step(10)
    import numpy as np
    e = _vel_err(g.fields(), o.fields())
    Fg, Fo = g.forces(0)[0], o.forces(0)[0]
    e["force_rel"] = float(np.abs(Fg - Fo).max() / max(np.abs(Fo).max(), 1e-300))
    e["steps"] = 10
    out["served_request_fp32_shifted"] = e
    g.close()
    return out


def plain_mlups(args, cases, lbmib, precision):
    """The members one at a time through the plain per-simulation path
    (direct launches, no batch, no graph)."""
    updates, seconds = 0, 0.0
    for c in cases[:args.fp64_sample]:
        s = lbmib.Sim.from_case(c, precision=precision)
        s.step(2)
        s.sync()
        t0 = time.perf_counter()
        s.step(args.fp64_steps)
        s.sync()
        seconds += time.perf_counter() - t0
        updates += c["nx"] * c["ny"] * args.fp64_steps
        s.close()
    return updates / seconds / 1e6, updates


def fp64_leg(args, cases, lbmib, wl, torch, np):
    """Plain FP64 and plain FP32 paths on the first members (one at a time,
    direct launches), the batched FP32 path on the same members, and the
    FP32-vs-FP64 velocity difference on a Couette member."""
    f64_mlups, f64_updates = plain_mlups(args, cases, lbmib, lbmib.F64)
    f32_plain_mlups, _ = plain_mlups(args, cases, lbmib, lbmib.F32_SHIFTED)
    # batched FP32 on the same sample, for a like-for-like speedup
    sample = [lbmib.Sim.from_case(c, precision=lbmib.F32_SHIFTED) for c in cases[:args.fp64_sample]]
    b2 = lbmib.Batch(lbmib.F32_SHIFTED)
    for s in sample:
        b2.admit(s)
    b2.step(10)  # captures the replayed graphs (1 and 8 steps) before the timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b2.step(args.fp64_steps)
    torch.cuda.synchronize()
    f32_sample_mlups = f64_updates / (time.perf_counter() - t0) / 1e6
    b2.close()
    del sample

    # ---- accuracy of the FP32 path against the FP64 path on one member (Couette 64)
    ref = wl.couette(64)
    a = lbmib.Sim.from_case(ref, precision=lbmib.F64)
    b = lbmib.Sim.from_case(ref, precision=lbmib.F32_SHIFTED)
    a.step(2000)
    b.step(2000)
    _, ua, va = a.fields()
    _, ub, vb = b.fields()
    err = float(np.sqrt(np.sum((ua - ub) ** 2 + (va - vb) ** 2) / np.sum(ua ** 2 + va ** 2)))

    return f64_mlups, f32_sample_mlups, err, f32_plain_mlups


def mrt_leg(args, cases, lbmib, wl, torch, tiling, lanes):
    """The same set with the MRT collision (rates of the validation cases) in
    every member: batched throughput and the sweep's per-launch duration."""
    sims = [lbmib.Sim.from_case(c, precision=lbmib.F32_SHIFTED, mrt_s=wl.mrt_rates(c["tau"])) for c in cases]
    b = lbmib.Batch(lbmib.F32_SHIFTED)
    for s in sims:
        assert b.admit(s)
    b.set_tiling(tiling)
    if lanes:
        b.set_lanes(lanes)
    b.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.mrt_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.set_lanes(1)
    ms, pcells = b.profile(10)
    b.close()
    del sims
    cells = sum(c["nx"] * c["ny"] for c in cases)
    sweep_ms = ms[0] / 10
    ach = SWEEP_BYTES_F32 * pcells / (sweep_ms * 1e-3) / 1e9
    return {"value": round(cells * args.mrt_steps / wall / 1e6, 1), "unit": "MLUPS", "steps": args.mrt_steps,
            "sweep_launch_ms": round(sweep_ms, 4), "sweep_achieved_gbs": round(ach, 1),
            "sweep_frac": round(ach / HBM_PEAK_GBS, 4), "tiling": tiling,
            "rates": "s_e 1.1, s_eps 1.25, s_q 1.8, s_nu 1/tau"}


def served_steady_leg(args, lbmib, wl, torch, steps):
    """The first eight requests of the overload leg stepped together with no
    arrivals or retirements: one lane, and two interleaved halves of equal
    node count (lane mode 4), whose corrections run beside each other's
    sweeps."""
    arr = wl.arrivals(seed=args.seed + 1, rate=20.0, count=max(8, args.serve_overload), steps=10 * args.serve_steps)
    cases = [r["case"] for r in arr[:8]]
    cells = sum(c["nx"] * c["ny"] for c in cases)
    sims = [lbmib.Sim.from_case(c, precision=lbmib.F32_SHIFTED) for c in cases]
    b = lbmib.Batch(lbmib.F32_SHIFTED)
    for s in sims:
        assert b.admit(s)
    out = {"requests": 8, "nodes": cells, "steps": steps}
    for lanes, key in ((1, "one_lane"), (4, "two_interleaved_halves")):
        b.set_lanes(lanes)
        b.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[key] = {"mlups": round(cells * steps / wall / 1e6, 1), "ms_per_step": round(wall / steps * 1e3, 4)}
    b.close()
    for s in sims:
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--sims", type=int, default=256)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--fp64-sample", type=int, default=16)
    ap.add_argument("--fp64-steps", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="host time of the oracle sample, split between one thread and all threads")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the oracle on the other configurations (bounded steps; minutes)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="print the CPU baseline alone (with --cpu-configs: every configuration) and stop")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default sweep tiling instead of timing the candidates on the set")
    ap.add_argument("--tiling", type=int, default=-1)
    ap.add_argument("--lanes", type=int, default=0,
                    help="1, 2 (free-running), 3 (interleaved heavy/light) or 4 (interleaved equal halves) "
                         "to request the batch's lanes (default 0: the autotuner times the heavy/light split, "
                         "equal halves and one lane under every tiling and keeps the fastest)")
    ap.add_argument("--mrt-steps", type=int, default=100,
                    help="timed steps of the same set with the MRT collision (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-steps", type=int, default=2000)
    ap.add_argument("--serve-overload", type=int, default=16,
                    help="requests of the overload leg (10x the steps, HBM budget of 8 requests; 0 skips it)")
    ap.add_argument("--served-steady-steps", type=int, default=200,
                    help="steps of the served steady-state leg (0 skips it)")
    ap.add_argument("--only-served-steady", action="store_true",
                    help="run the served steady-state leg alone (for profiler runs)")
    ap.add_argument("--only-batch", action="store_true",
                    help="time the batched set only (for profiler runs): no CPU baseline, FP64 sample, "
                         "accuracy or serving legs")
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(json.loads(args.cpu_worker))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every simulation of the set fits one MI355X and the set "
              "shards by simulation with no communication; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    from paper_1803_09380_amd import workloads as wl
    if args.only_served_steady:
        import torch
        from paper_1803_09380_amd import lbmib
        torch.cuda.init()
        print(json.dumps({"served_steady": served_steady_leg(args, lbmib, wl, torch, args.served_steady_steps)}),
              flush=True)
        return
    cases = wl.batch(seed=args.seed, count=args.sims, precision=wl.F32)

    if args.only_batch:
        args.served_steady_steps = 0
        args.no_cpu = True
        args.fp64_sample = 0
        args.serve_requests = 0
        args.serve_overload = 0
        args.mrt_steps = 0
    cpu = None
    if not args.no_cpu:
        cpu = run_cpu_baseline(args)
        if args.cpu_only:
            print(json.dumps({"cpu_baseline": cpu}), flush=True)
            return

    import numpy as np
    import torch
    from paper_1803_09380_amd import lbmib

    torch.cuda.init()
    cells = sum(c["nx"] * c["ny"] for c in cases)
    markers = sum(b["n"] for c in cases for b in c["bodies"])

    # ---- FP32 shifted, batched
    sims = [lbmib.Sim.from_case(c, precision=lbmib.F32_SHIFTED) for c in cases]
    batch = lbmib.Batch(lbmib.F32_SHIFTED)
    for s in sims:
        assert batch.admit(s)
    if args.tiling >= 0:
        batch.set_tiling(args.tiling)
    if args.lanes:
        batch.set_lanes(args.lanes)
    tiling = args.tiling
    if args.tiling < 0 and not args.no_autotune:
        tiling = batch.autotune(trials=20)
    lanes = batch.lanes
    lane_mode = batch.lane_mode
    batch.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    mlups = cells * args.steps / wall / 1e6

    # ---- per-kernel durations on the batch stream (HIP events), same tables and
    # grids; in one lane, so that one sweep launch covers every node
    if lanes != 1:
        batch.set_lanes(1)
    ms, pcells = batch.profile(args.profile_steps)
    sweep_ms = ms[0] / args.profile_steps
    achieved = SWEEP_BYTES_F32 * pcells / (sweep_ms * 1e-3) / 1e9
    in_use = tiling if tiling >= 0 else batch.tiling
    traffic = sweep_traffic(in_use)
    unstable = 0
    for s in sims:
        try:
            s.sync()
        except lbmib.LbmError as e:
            if e.code == lbmib.ERR_UNSTABLE:
                unstable += 1
            else:
                raise
    batch.close()
    del sims
    torch.cuda.synchronize()

    # ---- the same set with the MRT collision
    mrt = None
    if args.mrt_steps > 0:
        mrt = mrt_leg(args, cases, lbmib, wl, torch, in_use, args.lanes)

    # ---- FP64 plain path: members of the same set one at a time, direct launches
    f64_mlups = f32_sample_mlups = err = f32_plain_mlups = None
    f64_updates, f64_time = 0, 0.0
    if args.fp64_sample > 0:
        f64_mlups, f32_sample_mlups, err, f32_plain_mlups = fp64_leg(args, cases, lbmib, wl, torch, np)

    # ---- served stream: Poisson arrivals of settling requests, continuous batching
    serving = None
    if args.serve_requests > 0:
        from paper_1803_09380_amd.serve import GpuExecutor, Request, Server
        arr = wl.arrivals(seed=args.seed, rate=20.0, count=args.serve_requests, steps=args.serve_steps)
        reqs = [Request(rid=r["id"], t_arrive=r["t_arrive"], case=r["case"], steps=r["steps"]) for r in arr]
        budget = 64 << 30
        ex = GpuExecutor(lbmib.F32_SHIFTED, hbm_budget=budget)
        srv = Server(ex, hbm_budget=budget, chunk=100)
        srv.run(reqs)
        ex.close()
        serving = srv.stats.summary()
        serving["frac_of_peak"] = frac_of_peak(serving["aggregate_mlups"])
        serving.update({"arrivals": "Poisson, mean 20/s, seed %d" % args.seed, "lattice": "400x4000 closed box",
                        "steps_per_request": args.serve_steps, "hbm_budget_bytes": budget,
                        "particles": "1 or 2 free circles, D 16..40, density ratio 1.01..1.5",
                        "lanes": "two interleaved halves while at least %d requests are on the device" % ex.halves_from})

    # ---- overload: ten times the steps per request and an HBM budget of eight
    # requests, so that arrivals queue for admission
    overload = None
    if args.serve_overload > 0:
        from paper_1803_09380_amd.serve import GpuExecutor, Request, Server
        arr = wl.arrivals(seed=args.seed + 1, rate=20.0, count=args.serve_overload, steps=10 * args.serve_steps)
        reqs = [Request(rid=r["id"], t_arrive=r["t_arrive"], case=r["case"], steps=r["steps"]) for r in arr]
        probe = lbmib.Sim.from_case(arr[0]["case"], precision=lbmib.F32_SHIFTED)
        budget = 8 * probe.device_bytes + probe.device_bytes // 2
        probe.close()
        ex = GpuExecutor(lbmib.F32_SHIFTED, hbm_budget=budget)
        srv = Server(ex, hbm_budget=budget, chunk=100)
        srv.run(reqs)
        ex.close()
        overload = srv.stats.summary()
        overload["frac_of_peak"] = frac_of_peak(overload["aggregate_mlups"])
        overload.update({"arrivals": "Poisson, mean 20/s, seed %d" % (args.seed + 1),
                         "lattice": "400x4000 closed box", "steps_per_request": 10 * args.serve_steps,
                         "hbm_budget_bytes": budget, "budget_requests": 8,
                         "lanes": "two interleaved halves while at least %d requests are on the device" % ex.halves_from})

    # ---- the overload leg's mix in steady state, one lane and two interleaved halves
    served_steady = None
    if args.served_steady_steps > 0:
        served_steady = served_steady_leg(args, lbmib, wl, torch, args.served_steady_steps)

    # ---- measured HBM copy (hand-written 16-byte copies and torch's) beside the datasheet peak
    copy = None
    if not args.only_batch:
        import copy_probe
        copy = copy_probe.measure(mib=1024, reps=10)

    # ---- CPU-baseline leg, second part: every GPU path against the FP64 oracle
    vs_oracle = None
    if cpu is not None:
        vs_oracle = oracle_errors(cases, lbmib, wl)
        cpu["gpu_vs_oracle"] = vs_oracle

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched uneven set: %d seeded simulations (Couette side 64..512 or cylinder "
                        "channel 20Dx10D with D 16..64, Re 10..100), FP32 shifted populations, "
                        "10 correction sweeps per step" % args.sims,
            "seed": args.seed, "sims": args.sims, "cells": cells, "markers": markers,
            "tiling": in_use, "lanes": lanes, "lane_mode": lane_mode,
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "traffic_over_algorithmic": None if traffic is None else round(traffic / (SWEEP_BYTES_F32 * pcells), 3),
            "measured_copy_gbs": None if copy is None else copy["best_copy_gbs"],
            "measured_copy": None if copy is None else copy["best_copy"],
            "frac_of_measured_copy": None if copy is None else round(achieved / copy["best_copy_gbs"], 4),
            "torch_copy_gbs": None if copy is None else round(copy["torch_copy_gbs"], 1),
            "step_frac": frac_of_peak(mlups),
            "step_frac_note": "whole step (sweep, boundary, correction, bookkeeping) at 72 B per node update",
            "kernel": "k_sweep<float>", "launch_ms": round(sweep_ms, 4),
            "bytes_per_cell": SWEEP_BYTES_F32, "cells_per_launch": pcells,
            "step_split_ms": {"sweep": round(ms[0] / args.profile_steps, 4),
                              "boundary": round(ms[1] / args.profile_steps, 4),
                              "correction": round(ms[2] / args.profile_steps, 4),
                              "bookkeeping": round(ms[3] / args.profile_steps, 4)},
        },
        "fp64_plain": None if f64_mlups is None else {
            "value": round(f64_mlups, 1), "unit": "MLUPS",
            "sample": "first %d members, %d steps each, one at a time" % (args.fp64_sample, args.fp64_steps),
            "fp32_batched_same_sample": round(f32_sample_mlups, 1),
            "speedup_fp32_batched": round(f32_sample_mlups / f64_mlups, 2),
            "fp32_plain_same_sample": round(f32_plain_mlups, 1),
            "speedup_of_batching_fp32": round(f32_sample_mlups / f32_plain_mlups, 2)},
        "accuracy": None if err is None else {"fp32_vs_fp64_velocity_rel_l2": err, "case": "couette64, 2000 steps",
                                              "vs_fp64_oracle": vs_oracle},
        "mrt": mrt,
        "unstable_members": unstable,
        "serving": serving,
        "serving_overload": overload,
        "served_steady": served_steady,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
