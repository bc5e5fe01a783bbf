"""Runs the paper's own validation set-ups on the GPU and reports the quantities
the paper prints next to its values.

  python -m paper_1803_09380_amd.validate table1 [--re 20 40 100 200]
  python -m paper_1803_09380_amd.validate dkt
  python -m paper_1803_09380_amd.validate single [--ratios 1.0015 1.003 1.01 1.03]
  python -m paper_1803_09380_amd.validate tgv [--sizes 10 20 40 80]
  python -m paper_1803_09380_amd.validate couette [--grids 32 64 128 256 512]
  python -m paper_1803_09380_amd.validate cylinder [--re 20 40 100]

Every case runs through the library (batched FP32 shifted populations unless
--f64); diagnostics are host-side post-processing of the returned fields,
forces and body states.  Prints one JSON object.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import diagnostics as dg
from . import workloads as wl

# Table 1, row "Present" (Sec. 3.2): C_d, L_w/D, separation angle for Re 20 and
# 40; C_d, C_l amplitude and St for Re 100 and 200.
TABLE1_PAPER = {
    20: {"cd": 2.181, "lw_over_d": 0.987, "theta_deg": 44.2},
    40: {"cd": 1.643, "lw_over_d": 2.46, "theta_deg": 53.2},
    100: {"cd": 1.415, "cl": 0.358, "st": 0.166},
    200: {"cd": 1.405, "cl": 0.719, "st": 0.196},
}
# Sec. 3.3.2: the gap starts closing, the pair kisses, the pair separates (s).
DKT_PAPER = {"drafting": 0.514, "kissing": 1.326, "tumbling": 2.492}


def _precision(lbmib, f64):
    return lbmib.F64 if f64 else lbmib.F32_SHIFTED


def _run_batch(lbmib, cases, budgets, sample, f64, record):
    """Admit the cases into one batch with their step budgets, advance in
    chunks of `sample` steps and call record(k, sim, step) for each live
    member after every chunk.  Returns the sims (synchronised)."""
    prec = _precision(lbmib, f64)
    sims = [lbmib.Sim.from_case(c, precision=prec) for c in cases]
    b = lbmib.Batch(prec)
    for s, n in zip(sims, budgets):
        assert b.admit(s, steps=n)
    done = 0
    while done < max(budgets):
        n = min(sample, max(budgets) - done)
        b.step(n)
        b.sync()
        done += n
        for k, s in enumerate(sims):
            if done <= budgets[k]:
                record(k, s, done)
    b.close()
    return sims


def table1(lbmib, res, f64=False, D=40.0, steady_steps=None, unsteady_steps=None, sample=20, periods=8,
           dump=None, U0=0.1, sides=wl.FREESLIP, outlet=wl.PRESSURE, window=None, field_every=None):
    """Flow past a cylinder at the Reynolds numbers of Table 1.

    Steady cases (Re < 49) report the drag averaged over the last `window`
    steps and L_w, separation angle from the velocity field averaged over
    snapshots `field_every` steps apart in that window: acoustic waves
    reflected between inlet and outlet persist for a long time at these
    viscosities and make single snapshots noisy.  Unsteady cases report the
    mean drag, lift amplitude and Strouhal number over the last `periods`
    shedding periods.  With `dump` (a path prefix) the force histories and
    the velocity field around the body are written to <dump>_Re<Re>.npz."""
    conv = D / U0  # steps per D/U0
    steady_steps = steady_steps or int(200 * conv)
    unsteady_steps = unsteady_steps or int(400 * conv)
    window = window or int(20 * conv)
    field_every = field_every or int(conv)
    assert field_every % sample == 0
    cases = [wl.table1_cylinder(Re, D=D, U0=U0, precision=wl.F64 if f64 else wl.F32, sides=sides, outlet=outlet)
             for Re in res]
    budgets = [steady_steps if Re < 49 else unsteady_steps for Re in res]
    hist = [[] for _ in res]
    acc = [[0, 0.0, 0.0] for _ in res]

    def record(k, s, step):
        F = s.forces(0)[0]
        cd, cl = dg.force_coefficients(F, U0, D)
        hist[k].append((step, cd, cl))
        if k == 0 and step % 20000 == 0:
            print("table1: %d steps" % step, file=sys.stderr, flush=True)
        if res[k] < 49 and step > budgets[k] - window and step % field_every == 0:
            _, ux, uy = s.fields()
            acc[k][0] += 1
            acc[k][1] = acc[k][1] + ux
            acc[k][2] = acc[k][2] + uy

    t0 = time.perf_counter()
    sims = _run_batch(lbmib, cases, budgets, sample, f64, record)
    wall = time.perf_counter() - t0
    out = {}
    for Re, s, c, h, a in zip(res, sims, cases, hist, acc):
        h = np.array(h)
        xc, yc = c["bodies"][0]["xc"]
        R = c["bodies"][0]["radius"]
        r = {"steps": int(h[-1, 0]), "paper": TABLE1_PAPER.get(Re)}
        rho, ux, uy = s.fields()
        if dump:
            x0, x1 = int(xc - 2 * D), int(xc + 6 * D)
            y0, y1 = int(yc - 2 * D), int(yc + 2 * D)
            np.savez_compressed("%s_Re%g.npz" % (dump, Re), hist=h, ux=ux[y0:y1, x0:x1], uy=uy[y0:y1, x0:x1],
                                rho=rho[y0:y1, x0:x1], origin=np.array([x0, y0]), centre=np.array([xc, yc]), R=R)
        if Re < 49:
            mu, mv = a[1] / a[0], a[2] / a[0]
            win = h[:, 0] > h[-1, 0] - window
            up, lo = dg.separation_angles(mu, mv, xc, yc, R, offset=1.0)
            th0, ths = dg.separation_angle_at_surface(mu, mv, xc, yc, R)
            r.update({"cd": float(h[win, 1].mean()), "cl": float(h[win, 2].mean()),
                      "cd_oscillation": float(0.5 * (h[win, 1].max() - h[win, 1].min())),
                      "averaged_over_steps": int(window), "field_snapshots": a[0],
                      "lw_over_d": dg.recirculation_length(mu, xc, yc, R) / D,
                      "lw_over_d_last_snapshot": dg.recirculation_length(ux, xc, yc, R) / D,
                      "theta_deg": th0, "theta_at_offset_1": 0.5 * (up + lo), "theta_upper_lower_offset_1": [up, lo],
                      "theta_offsets_1_to_3": ths})
        else:
            sh = dg.shedding(h[len(h) // 2:, 0], h[len(h) // 2:, 2], h[len(h) // 2:, 1], periods=periods)
            if sh is None:
                r.update({"cd": float(h[-1, 1]), "cl": None, "st": None, "note": "no shedding found"})
            else:
                r.update({"cd": sh["cd_mean"], "cl": sh["cl_amplitude"],
                          "st": dg.strouhal(sh["period"], D, U0), "periods_used": sh["cycles"]})
        if r["paper"]:
            r["rel_diff"] = {k: (r[k] - v) / v for k, v in r["paper"].items() if r.get(k) is not None}
        out[str(Re)] = r
        s.close()
    return {"case": "table1", "precision": "f64" if f64 else "f32_shifted", "D": D, "U0": U0,
            "sides": {wl.FREESLIP: "free slip", wl.PERIODIC: "periodic", wl.WALL: "wall"}[sides],
            "outlet": {wl.PRESSURE: "non-equilibrium extrapolation at rho0", wl.OUTFLOW: "zero gradient"}[outlet],
            "wall_s": wall, "results": out}


def dkt(lbmib, f64=False, seconds=4.0, sample=5):
    case = wl.dkt_pair(precision=wl.F64 if f64 else wl.F32)
    dt = case["meta"]["units"]["dt"]
    steps = int(round(seconds / dt))
    rows = []

    def record(k, s, step):
        a = s.forces(0)[3]
        b = s.forces(1)[3]
        rows.append([step * dt, a[0], a[1], b[0], b[1], math.hypot(a[0] - b[0], a[1] - b[1])])

    t0 = time.perf_counter()
    sims = _run_batch(lbmib, [case], [steps], sample, f64, record)
    wall = time.perf_counter() - t0
    sims[0].close()
    h = np.array(rows)
    ev = dg.dkt_events(h[:, 0], h[:, 5], case["meta"]["D"])
    return {"case": "dkt", "precision": "f64" if f64 else "f32_shifted", "steps": steps, "dt_s": dt,
            "events_s": ev, "paper_s": DKT_PAPER,
            "rel_diff": {k: (ev[k] - v) / v for k, v in DKT_PAPER.items() if ev[k] is not None},
            "min_distance_over_d": float(h[:, 5].min() / case["meta"]["D"]), "wall_s": wall,
            "history_every_s": float(h[1, 0] - h[0, 0]),
            "distance_over_d_every_0.1s": [float(v) for v in
                                           h[::max(1, int(round(0.1 / (h[1, 0] - h[0, 0])))), 5] / case["meta"]["D"]]}


def single(lbmib, ratios, f64=False, seconds=2.0, sample=50):
    cases = [wl.single_particle_channel(r, precision=wl.F64 if f64 else wl.F32) for r in ratios]
    dt = cases[0]["meta"]["units"]["dt"]
    steps = int(round(seconds / dt))
    hist = [[] for _ in ratios]

    def record(k, s, step):
        st = s.forces(0)[3]
        hist[k].append([step * dt, st[0], st[1], st[2], st[3], st[4]])

    t0 = time.perf_counter()
    sims = _run_batch(lbmib, cases, [steps] * len(cases), sample, f64, record)
    wall = time.perf_counter() - t0
    out = {}
    for r, c, h, s in zip(ratios, cases, hist, sims):
        h = np.array(h)
        W, cl = c["meta"]["W"], c["meta"]["centre_line"]
        lateral = (h[:, 2] - cl) / W
        vy = h[:, 4]
        sgn = np.sign(vy[np.abs(vy) > 1e-7])
        out[str(r)] = {"final_offset_over_w": float(lateral[-1]), "start_offset_over_w": float(lateral[0]),
                       "max_crossing_over_w": float(-lateral.min()) if lateral[0] > 0 else float(lateral.max()),
                       "lateral_velocity_sign_changes": int(np.count_nonzero(np.diff(sgn))),
                       "settling_velocity_cm_s": float(h[-1, 3] * c["meta"]["units"]["dx"] / dt),
                       "fallen_over_d": float((h[-1, 1] - h[0, 1]) / c["meta"]["D"])}
        s.close()
    return {"case": "single", "precision": "f64" if f64 else "f32_shifted", "seconds": seconds, "steps": steps,
            "wall_s": wall, "results": out}


def tgv_run(sim, case, steps=None):
    """Drive a Taylor-Green case (workloads.tgv_cylinder) on any simulation
    object with set_fields / set_boundary_velocity / set_marker_velocities /
    step / fields: start from the equilibrium of the analytic field at t = 0,
    before step n + 1 set the box and marker velocities of t = n + 1, and
    return the L2 velocity error of Eq. 31 over all nodes at the end
    (t* = 1 by default)."""
    steps = case["meta"]["steps"] if steps is None else steps
    rho, ux, uy = wl.tgv_solution(case, 0.0)
    sim.set_fields(rho, ux, uy)
    has_body = len(case["bodies"]) > 0
    for n in range(steps):
        t = float(n + 1)
        sim.set_boundary_velocity(wl.tgv_boundary(case, t))
        if has_body:
            sim.set_marker_velocities(0, wl.tgv_markers(case, t))
        sim.step(1)
    _, gx, gy = sim.fields()
    _, ax, ay = wl.tgv_solution(case, float(steps))
    return {"steps": steps, "l2": float(np.sqrt(np.mean((gx - ax) ** 2 + (gy - ay) ** 2))),
            "u0": case["meta"]["u0"]}


def tgv(lbmib, sizes, f64=True, cylinder=True):
    """L2 error of the Taylor-Green vortex with a cylinder at t* = 1 (Sec. 3.1.1)
    for box half-widths L (the cylinder's diameter), and the observed orders."""
    out = {}
    t0 = time.perf_counter()
    for L in sizes:
        case = wl.tgv_cylinder(L, precision=wl.F64 if f64 else wl.F32, cylinder=cylinder)
        s = lbmib.Sim.from_case(case)
        out[str(L)] = tgv_run(s, case)
        s.close()
    errs = [out[str(L)]["l2"] for L in sizes]
    orders = [math.log(errs[k] / errs[k + 1]) / math.log(sizes[k + 1] / sizes[k]) for k in range(len(sizes) - 1)]
    return {"case": "tgv", "cylinder": cylinder, "precision": "f64" if f64 else "f32_shifted",
            "results": out, "orders": orders, "wall_s": time.perf_counter() - t0}


def couette(lbmib, sides, steps_per_k2=3000):
    """Cylindrical Couette flow (Sec. 3.1.2) on the workloads' geometry at each
    side (k = side / 64; R1 = 12k, R2 = 24k, wall speed 0.01/k, tau = 0.8, so
    Re is fixed), steps_per_k2 * k^2 steps, in FP64 and FP32 batches.  Reports
    the relative annulus error, the absolute L2 norm of Eq. 35 on theta = pi/2,
    their observed orders, the inner torque against the closed form, the mass
    drift and the FP32-FP64 velocity difference."""
    cases = [wl.couette(sd, precision=wl.F64) for sd in sides]
    budgets = [int(steps_per_k2 * (sd / 64.0) ** 2) for sd in sides]
    out = {"case": "couette", "sides": list(sides), "steps": budgets, "precisions": {}}
    fields = {}
    t0 = time.perf_counter()
    for name, f64 in (("f64", True), ("f32_shifted", False)):
        def progress(k, s, step):
            if k == 0:
                print("couette %s: %d steps" % (name, step), file=sys.stderr, flush=True)

        sims = _run_batch(lbmib, cases, budgets, 20000, f64, progress)
        rows = []
        for c, s in zip(cases, sims):
            m = c["meta"]
            rho, ux, uy = s.fields()
            fields[(name, c["nx"])] = (ux, uy)
            rel, e35 = dg.couette_errors(ux, uy, m["centre"], m["R1"], m["R2"], m["omega1"])
            T = s.forces(1)[1]
            Ta = dg.couette_torque(m["nu"] * c["rho0"], m["omega1"], m["R1"], m["R2"])
            rows.append({"side": c["nx"], "rel_l2": rel, "l2_eq35": e35, "l2_eq35_relative": e35 / (m["omega1"] * m["R1"]),
                         "torque_over_closed_form": T / Ta,
                         "mass_drift": float(rho.sum() / (c["rho0"] * c["nx"] * c["ny"]) - 1.0)})
            s.close()
        out["precisions"][name] = {
            "rows": rows,
            "order_rel_l2": -dg.observed_order(sides, [r["rel_l2"] for r in rows]) if len(rows) > 1 else None,
            "order_eq35_lattice_units": -dg.observed_order(sides, [r["l2_eq35"] for r in rows]) if len(rows) > 1 else None,
            "order_eq35_relative": -dg.observed_order(sides, [r["l2_eq35_relative"] for r in rows]) if len(rows) > 1 else None}
    out["fp32_vs_fp64_velocity_rel_l2"] = {}
    out["fp32_vs_fp64_velocity_max_rel"] = {}
    for c in cases:
        a, b = fields[("f32_shifted", c["nx"])], fields[("f64", c["nx"])]
        num = np.sum((a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2)
        den = np.sum(b[0] ** 2 + b[1] ** 2)
        out["fp32_vs_fp64_velocity_rel_l2"][str(c["nx"])] = float(np.sqrt(num / den))
        mx = max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max())
        out["fp32_vs_fp64_velocity_max_rel"][str(c["nx"])] = float(mx / max(np.abs(b[0]).max(), np.abs(b[1]).max()))
    out["wall_s"] = time.perf_counter() - t0
    return out


COUETTE_PAPER_SETS = [(0.5, 0.65), (0.5, 0.85), (0.8, 0.65), (0.8, 0.85)]  # (radius ratio R, tau_s)


def couette_paper(lbmib, grids, f64=True, sets=COUETTE_PAPER_SETS):
    """Cylindrical Couette flow as set up in Sec. 3.1.2 (workloads.couette_paper:
    MRT, Re = 10, tau_s = 0.65 / 0.85, R = 0.5 / 0.8, outer radius on N lattice
    spacings), every grid and set in one batch, each run to its steady state.
    Reports per set the Eq. 35 norm in lattice units and relative to the wall
    speed U1, the relative error over the annulus, and the least-squares order
    of each in 1/N.  Refinement keeps tau_s and Re, so U1 ~ 1/N and the
    lattice-unit norm gains one order over the scale-free relative one."""
    cases = [wl.couette_paper(N, r, t, precision=wl.F64 if f64 else wl.F32) for (r, t) in sets for N in grids]
    budgets = [c["meta"]["steps"] for c in cases]

    def progress(k, s, step):
        if k == 0 and step % 20000 == 0:
            print("couette_paper: %d steps" % step, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    sims = _run_batch(lbmib, cases, budgets, 4000, f64, progress)
    out = {"case": "couette_paper", "grids": list(grids), "precision": "f64" if f64 else "f32_shifted", "sets": []}
    h = [1.0 / N for N in grids]
    for j, (r, t) in enumerate(sets):
        rows = []
        for i, N in enumerate(grids):
            c, sim = cases[j * len(grids) + i], sims[j * len(grids) + i]
            m = c["meta"]
            _, ux, uy = sim.fields()
            rel, e35 = dg.couette_errors(ux, uy, m["centre"], m["R1"], m["R2"], m["omega1"])
            rows.append({"N": N, "steps": m["steps"], "eq35_lattice": e35, "eq35_relative": e35 / m["U1"],
                         "annulus_relative": rel})
            sim.close()
        order = lambda key: dg.observed_order(h, [q[key] for q in rows]) if len(rows) > 1 else None
        out["sets"].append({"R": r, "tau_s": t, "rows": rows, "order_eq35_lattice": order("eq35_lattice"),
                            "order_eq35_relative": order("eq35_relative"),
                            "order_annulus_relative": order("annulus_relative")})
    out["wall_s"] = time.perf_counter() - t0
    return out


def cylinder_channel(lbmib, res, steps=None, sample=20, periods=8):
    """Flow past a fixed cylinder in a 1600 x 800 channel (D = 40 at (400, 400),
    126 markers, inflow U = 0.05, zero-gradient outflow, free-slip sides, BGK,
    FP32 shifted populations), all Reynolds numbers in one batch.  Reports C_d
    and C_l (mean and amplitude over the last shedding periods when the flow
    sheds), the largest normal velocity at the markers from the final field
    (non-penetration), and the batch's MLUPS."""
    D, U = 40.0, 0.05
    conv = D / U
    cases = [wl.cylinder(nx=1600, ny=800, D=D, centre=(400.0, 400.0), U=U, Re=Re) for Re in res]
    budgets = [steps or (int(100000) if Re < 49 else int(300000)) for Re in res]
    hist = [[] for _ in res]

    def record(k, s, step):
        F = s.forces(0)[0]
        cd, cl = dg.force_coefficients(F, U, D)
        hist[k].append((step, cd, cl))
        if k == 0 and step % 20000 == 0:
            print("cylinder: %d steps" % step, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    sims = _run_batch(lbmib, cases, budgets, sample, False, record)
    wall = time.perf_counter() - t0
    cells = sum(c["nx"] * c["ny"] * n for c, n in zip(cases, budgets))
    out = {}
    for Re, s, c, h in zip(res, sims, cases, hist):
        h = np.array(h)
        b = c["bodies"][0]
        _, ux, uy = s.fields()
        xy = b["xy"]
        nrm = (xy - np.array(b["xc"])) / b["radius"]
        un = dg.bilinear(ux, xy[:, 0], xy[:, 1]) * nrm[:, 0] + dg.bilinear(uy, xy[:, 0], xy[:, 1]) * nrm[:, 1]
        r = {"steps": int(h[-1, 0]), "max_normal_velocity_over_U": float(np.abs(un).max() / U),
             "max_slip_after_sweeps_over_U": float(s.forces(0)[2][1] / U)}
        sh = dg.shedding(h[len(h) // 2:, 0], h[len(h) // 2:, 2], h[len(h) // 2:, 1], periods=periods) if Re >= 49 else None
        if sh is None:
            win = h[:, 0] > h[-1, 0] - 20 * conv
            r.update({"cd": float(h[win, 1].mean()), "cl": float(h[win, 2].mean())})
        else:
            r.update({"cd": sh["cd_mean"], "cl_amplitude": sh["cl_amplitude"], "st": dg.strouhal(sh["period"], D, U)})
        out[str(Re)] = r
        s.close()
    return {"case": "cylinder_channel", "precision": "f32_shifted", "results": out, "wall_s": wall,
            "mlups_including_host_sampling": cells / wall / 1e6}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("case", choices=["table1", "dkt", "single", "tgv", "couette", "couette_paper", "cylinder"])
    ap.add_argument("--grids", type=int, nargs="+", default=[32, 64, 128, 256, 512],
                    help="Couette box sides (couette)")
    ap.add_argument("--steps-per-k2", type=int, default=3000)
    ap.add_argument("--sizes", type=int, nargs="+", default=[10, 20, 40, 80])
    ap.add_argument("--no-cylinder", action="store_true")
    ap.add_argument("--re", type=float, nargs="+", default=[20, 40, 100, 200])
    ap.add_argument("--ratios", type=float, nargs="+", default=[1.0015, 1.003, 1.01, 1.03])
    ap.add_argument("--f64", action="store_true")
    ap.add_argument("--f32", action="store_true", help="FP32 shifted populations (couette_paper)")
    ap.add_argument("--seconds", type=float, default=None)
    ap.add_argument("--steady-steps", type=int, default=None)
    ap.add_argument("--unsteady-steps", type=int, default=None)
    ap.add_argument("--dump", default=None, help="path prefix for .npz histories and fields (table1)")
    ap.add_argument("--u0", type=float, default=0.1, help="inflow speed (table1)")
    ap.add_argument("--sides", choices=["freeslip", "periodic"], default="freeslip",
                    help="south/north boundaries (table1)")
    ap.add_argument("--outlet", choices=["pressure", "outflow"], default="pressure",
                    help="east boundary (table1)")
    args = ap.parse_args(argv)
    from . import lbmib
    lbmib.load()
    if args.case == "table1":
        res = [int(r) if float(r).is_integer() else r for r in args.re]
        out = table1(lbmib, res, f64=args.f64, steady_steps=args.steady_steps, unsteady_steps=args.unsteady_steps,
                     dump=args.dump, U0=args.u0, sides={"freeslip": wl.FREESLIP, "periodic": wl.PERIODIC}[args.sides],
                     outlet={"pressure": wl.PRESSURE, "outflow": wl.OUTFLOW}[args.outlet])
    elif args.case == "dkt":
        out = dkt(lbmib, f64=args.f64, seconds=args.seconds or 4.0)
    elif args.case == "single":
        out = single(lbmib, args.ratios, f64=args.f64, seconds=args.seconds or 2.0)
    elif args.case == "tgv":
        out = tgv(lbmib, args.sizes, f64=True, cylinder=not args.no_cylinder)
    elif args.case == "couette":
        out = couette(lbmib, args.grids, steps_per_k2=args.steps_per_k2)
    elif args.case == "couette_paper":
        grids = args.grids if args.grids != [32, 64, 128, 256, 512] else [20, 40, 80, 160]
        out = couette_paper(lbmib, grids, f64=not args.f32)
    else:
        res = [int(r) if float(r).is_integer() else r for r in (args.re if args.re != [20, 40, 100, 200] else [20, 40, 100])]
        out = cylinder_channel(lbmib, res, steps=args.steady_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
