"""Seeded synthetic inputs with the shapes of the paper's test cases.

This module only describes problems: lattice sizes, relaxation times, boundary
types, and the Lagrangian markers of circles (the discretised interface Gamma
of Sec. 2.2).  It holds none of the method's arithmetic, so both the CPU
oracle and the GPU library can take their inputs from it.

Cases (lattice units):
  * cylindrical Couette flow (Sec. 3.1.2, Eqs. 32-34): periodic box of side s,
    k = s/64, outer circle R2 = 24k fixed, inner circle R1 = 12k turning
    counter-clockwise at tangential speed 0.01/k, tau = 0.8, markers about one
    lattice spacing apart (N = round(2 pi R)), Delta s = 2 pi R / N;
  * flow past a fixed cylinder (Sec. 3.2): channel, uniform inflow U at the west
    side, zero-gradient outflow at the east side, free-slip south/north, tau from
    Re = U D / nu;
  * settling particles (Sec. 3.3): closed box with walls, one or two free circles;
  * the paper's own set-ups: Table 1's cylinder (Sec. 3.2), the single particle
    in a channel (Sec. 3.3.1) and the DKT pair (Sec. 3.3.2).

A case may carry "mrt_s", the nine MRT rates (absent or None: BGK).
"""
import math

import numpy as np

PERIODIC, WALL, FREESLIP, VELOCITY, OUTFLOW, PRESSURE, DIRICHLET = range(7)
FIXED, FREE = 0, 1
F64, F32 = 0, 1


def mrt_rates(tau):
    """Relaxation rates of Eq. 6 in the moment order of Eq. 5 as chosen for the
    validation cases of Sec. 4.1: s_e = 1.1, s_epsilon = 1.25, s_q = 1.8 and
    s_s = 1/tau; the conserved moments' rates (rho, j) do not act and are 1."""
    return [1.0, 1.1, 1.25, 1.0, 1.8, 1.0, 1.8, 1.0 / tau, 1.0 / tau]


def circle_markers(xc, yc, R, n, phase=0.0):
    """n markers on a circle, angle 2 pi l / n + phase, counter-clockwise."""
    a = phase + 2.0 * np.pi * np.arange(n) / n
    return np.stack([xc + R * np.cos(a), yc + R * np.sin(a)], axis=1)


def couette(side=64, tau=0.8, u_inner=None, precision=F64, ib_iters=10):
    """Cylindrical Couette flow between a fixed outer circle and a turning inner one."""
    k = side / 64.0
    R1, R2 = 12.0 * k, 24.0 * k
    c = side / 2.0
    U1 = 0.01 / k if u_inner is None else u_inner
    n1, n2 = int(round(2 * math.pi * R1)), int(round(2 * math.pi * R2))
    bodies = [
        dict(kind=FIXED, n=n2, xy=circle_markers(c, c, R2, n2), uv=None,
             ds=np.full(n2, 2 * math.pi * R2 / n2), xc=(c, c), U=(0.0, 0.0), omega=0.0,
             theta=0.0, radius=R2, rho_s=0.0),
        dict(kind=FIXED, n=n1, xy=circle_markers(c, c, R1, n1), uv=None,
             ds=np.full(n1, 2 * math.pi * R1 / n1), xc=(c, c), U=(0.0, 0.0), omega=U1 / R1,
             theta=0.0, radius=R1, rho_s=0.0),
    ]
    return dict(name="couette%d" % side, nx=side, ny=side, tau=tau, rho0=1.0,
                bc=(PERIODIC,) * 4, u_in=(0.0, 0.0), u_init=(0.0, 0.0), ib_iters=ib_iters,
                precision=precision, gravity=(0.0, 0.0), bodies=bodies,
                meta=dict(R1=R1, R2=R2, omega1=U1 / R1, centre=(c, c), nu=(tau - 0.5) / 3.0))


def couette_paper(N, radius_ratio, tau, Re=10.0, margin=4, precision=F64, ib_iters=10):
    """Cylindrical Couette flow as set up in Sec. 3.1.2: outer radius R2 = 1
    resolved by N lattice spacings (dx = 1/N), inner radius R1 = R R2 with the
    radius ratio R = 0.5 or 0.8, Re = U1 (R2 - R1) / nu = 10 with U1 = omega1 R1,
    tau_s = 0.65 or 0.85 and the MRT rates of Sec. 4.1.  Refinement keeps tau_s
    and Re, so the lattice wall speed U1 = Re nu / (R2 - R1) falls as 1/N.

    The box is periodic with `margin` nodes between the outer circle and its
    periodic image's stencil.  meta["steps"] is the run length: 1.5 diffusion
    times of the gap and one of the inner disc (R1^2 / nu), after which the
    slowest transients (decay rates about pi^2 nu / (R2 - R1)^2 and
    14.7 nu / R1^2) are below 1e-6 of their start."""
    R2 = float(N)
    R1 = radius_ratio * R2
    side = int(2 * (N + margin))
    c = side / 2.0
    nu = (tau - 0.5) / 3.0
    U1 = Re * nu / (R2 - R1)
    n1, n2 = int(round(2 * math.pi * R1)), int(round(2 * math.pi * R2))
    bodies = [
        dict(kind=FIXED, n=n2, xy=circle_markers(c, c, R2, n2), uv=None,
             ds=np.full(n2, 2 * math.pi * R2 / n2), xc=(c, c), U=(0.0, 0.0), omega=0.0,
             theta=0.0, radius=R2, rho_s=0.0),
        dict(kind=FIXED, n=n1, xy=circle_markers(c, c, R1, n1), uv=None,
             ds=np.full(n1, 2 * math.pi * R1 / n1), xc=(c, c), U=(0.0, 0.0), omega=U1 / R1,
             theta=0.0, radius=R1, rho_s=0.0),
    ]
    steps = int(math.ceil(max(1.5 * (R2 - R1) ** 2, R1 * R1) / nu))
    return dict(name="couette_paper_N%d_R%g_tau%g" % (N, radius_ratio, tau), nx=side, ny=side, tau=tau,
                rho0=1.0, bc=(PERIODIC,) * 4, u_in=(0.0, 0.0), u_init=(0.0, 0.0), ib_iters=ib_iters,
                precision=precision, gravity=(0.0, 0.0), bodies=bodies, mrt_s=mrt_rates(tau),
                meta=dict(R1=R1, R2=R2, omega1=U1 / R1, U1=U1, centre=(c, c), nu=nu, N=N,
                          radius_ratio=radius_ratio, steps=steps))


def cylinder(nx=1600, ny=800, D=40.0, centre=None, U=0.05, Re=20.0, precision=F32, ib_iters=10,
             n_markers=None):
    """Flow past a fixed circular cylinder in a channel."""
    nu = U * D / Re
    tau = 3.0 * nu + 0.5
    R = D / 2.0
    cx, cy = centre if centre is not None else (nx / 4.0, ny / 2.0)
    n = n_markers if n_markers is not None else int(round(math.pi * D))
    body = dict(kind=FIXED, n=n, xy=circle_markers(cx, cy, R, n), uv=np.zeros((n, 2)),
                ds=np.full(n, 2 * math.pi * R / n), xc=(cx, cy), U=(0.0, 0.0), omega=0.0,
                theta=0.0, radius=R, rho_s=0.0)
    return dict(name="cylinder_%dx%d_D%g_Re%g" % (nx, ny, D, Re), nx=nx, ny=ny, tau=tau, rho0=1.0,
                bc=(VELOCITY, OUTFLOW, FREESLIP, FREESLIP), u_in=(U, 0.0), u_init=(U, 0.0),
                ib_iters=ib_iters, precision=precision, gravity=(0.0, 0.0), bodies=[body],
                meta=dict(D=D, U=U, Re=Re, nu=nu))


def settling(nx=400, ny=4000, D=24.0, density_ratio=1.2, two=False, tau=0.8, u_ref=0.04,
             precision=F32, ib_iters=10, lower=None):
    """One or two free circles settling under gravity in a closed box.

    Gravity is g = u_ref^2 / ((rho_s/rho_f - 1) D), which keeps the settling
    speed near u_ref (Mach well below 0.1)."""
    R = D / 2.0
    g = u_ref * u_ref / ((density_ratio - 1.0) * D)
    x0, y0 = lower if lower is not None else (nx / 2.0, ny - 400.0)
    n = int(round(math.pi * D))
    bodies = [dict(kind=FREE, n=n, xy=None, uv=None, ds=None, xc=(x0, y0), U=(0.0, 0.0),
                   omega=0.0, theta=0.0, radius=R, rho_s=density_ratio)]
    if two:
        bodies.append(dict(kind=FREE, n=n, xy=None, uv=None, ds=None,
                           xc=(x0 + 0.01 * D, y0 + 2.0 * D), U=(0.0, 0.0), omega=0.0, theta=0.0,
                           radius=R, rho_s=density_ratio))
    return dict(name="settling_%dx%d_D%g_r%g_%s" % (nx, ny, D, density_ratio, "two" if two else "one"),
                nx=nx, ny=ny, tau=tau, rho0=1.0, bc=(WALL,) * 4, u_in=(0.0, 0.0),
                u_init=(0.0, 0.0), ib_iters=ib_iters, precision=precision, gravity=(0.0, -g),
                bodies=bodies, meta=dict(D=D, g=g, density_ratio=density_ratio))


def table1_cylinder(Re, D=40.0, U0=0.1, precision=F32, collision_mrt=True, ib_iters=10, sides=FREESLIP,
                    outlet=PRESSURE):
    """Flow past a fixed cylinder as set up for Table 1 (Sec. 3.2): domain
    40D x 20D, cylinder centre at (10D, 10D), delta_x = D/40 (D = 40 lattice
    units), inflow U0 = 0.1, inlet and outlet by non-equilibrium extrapolation
    (velocity at the inlet, density rho0 at the outlet), free-slip sides (the
    paper does not name them), MRT with the rates of Sec. 4.1 (tau_s from
    Re = U0 D / nu).  The start is uniform flow at U0."""
    nx, ny = int(round(40 * D)), int(round(20 * D))
    case = cylinder(nx=nx, ny=ny, D=D, centre=(10.0 * D, 10.0 * D), U=U0, Re=Re, precision=precision,
                    ib_iters=ib_iters)
    case["name"] = "table1_Re%g_D%g" % (Re, D)
    case["mrt_s"] = mrt_rates(case["tau"]) if collision_mrt else None
    case["bc"] = (case["bc"][0], outlet, sides, sides)
    return case


# Physical set-ups of the particle cases of Sec. 3.3 (CGS units) and their
# lattice units: delta_x from the particle resolution, delta_t from
# nu_lattice = (tau - 1/2)/3 = nu delta_t / delta_x^2, g_lattice = g delta_t^2 / delta_x.
def lattice_units(dx_cm, tau, nu_cm2s=0.01, g_cms2=980.0):
    nu_lu = (tau - 0.5) / 3.0
    dt = nu_lu * dx_cm * dx_cm / nu_cm2s
    return dict(dx=dx_cm, dt=dt, nu_lu=nu_lu, g_lu=g_cms2 * dt * dt / dx_cm)


def single_particle_channel(density_ratio, precision=F32, ib_iters=10, start_below_inlet=None):
    """A particle settling in a channel (Sec. 3.3.1): D = 0.1 cm resolved by 26
    lattice units, width W = 4D, height H = 400/13 D, tau = 0.6, fluid density
    1 g/cm^3, nu = 0.01 cm^2/s, |g| = 980 cm/s^2, released from rest 0.31 W from
    the centre line.  Zero velocity at the inlet and a free-stream outlet.

    Lattice orientation: the channel runs along x (gravity +x), inlet at the
    west side (velocity rule with U = 0), outlet at the east side
    (zero-gradient), side walls south/north.  The release height is not
    given; the particle starts one channel width below the inlet by default."""
    D = 26.0
    W, H = int(round(4 * D)), int(round(400.0 / 13.0 * D))
    lu = lattice_units(0.1 / D, 0.6)
    R = D / 2.0
    x0 = float(W) if start_below_inlet is None else float(start_below_inlet)
    centre_line = (W - 1) / 2.0  # walls half a spacing outside nodes 0 and W-1
    y0 = centre_line - 0.31 * W
    n = int(round(math.pi * D))
    body = dict(kind=FREE, n=n, xy=None, uv=None, ds=None, xc=(x0, y0), U=(0.0, 0.0), omega=0.0,
                theta=0.0, radius=R, rho_s=density_ratio)
    return dict(name="single_particle_r%g" % density_ratio, nx=H, ny=W, tau=0.6, rho0=1.0,
                bc=(VELOCITY, OUTFLOW, WALL, WALL), u_in=(0.0, 0.0), u_init=(0.0, 0.0),
                ib_iters=ib_iters, precision=precision, gravity=(lu["g_lu"], 0.0), bodies=[body],
                mrt_s=None, meta=dict(D=D, W=W, H=H, centre_line=centre_line, units=lu,
                                      density_ratio=density_ratio))


def dkt_pair(precision=F32, ib_iters=10):
    """Drafting-kissing-tumbling of two particles (Sec. 3.3.2): channel 2 cm x
    8 cm on 200 x 800 nodes (D = 0.2 cm on 20 nodes), tau = 0.8, particle
    density 1.01 g/cm^3, nu = 0.01 cm^2/s, |g| = 980 cm/s^2, closed box, lower
    particle at (1.0, 6.8) cm, upper at (0.999, 7.2) cm.  Node i sits at
    (i + 1/2) delta_x, so a position p cm is p/delta_x - 1/2 lattice units."""
    nx, ny, D = 200, 800, 20.0
    dx = 2.0 / nx
    lu = lattice_units(dx, 0.8)
    to_lu = lambda p: p / dx - 0.5
    n = int(round(math.pi * D))
    bodies = [dict(kind=FREE, n=n, xy=None, uv=None, ds=None, xc=(to_lu(1.0), to_lu(6.8)), U=(0.0, 0.0),
                   omega=0.0, theta=0.0, radius=D / 2, rho_s=1.01),
              dict(kind=FREE, n=n, xy=None, uv=None, ds=None, xc=(to_lu(0.999), to_lu(7.2)), U=(0.0, 0.0),
                   omega=0.0, theta=0.0, radius=D / 2, rho_s=1.01)]
    return dict(name="dkt_200x800", nx=nx, ny=ny, tau=0.8, rho0=1.0, bc=(WALL,) * 4, u_in=(0.0, 0.0),
                u_init=(0.0, 0.0), ib_iters=ib_iters, precision=precision, gravity=(0.0, -lu["g_lu"]),
                bodies=bodies, mrt_s=None, meta=dict(D=D, units=lu))


def perimeter_nodes(nx, ny):
    """(x, y) of the perimeter nodes of a box in the order the prescribed
    velocities are given: south row, north row, west column, east column."""
    xs = list(range(nx))
    pts = [(x, 0) for x in xs] + [(x, ny - 1) for x in xs]
    pts += [(0, y) for y in range(1, ny - 1)] + [(nx - 1, y) for y in range(1, ny - 1)]
    return np.array(pts, dtype=np.float64)


def tgv_cylinder(L, precision=F64, tau=0.65, Re=10.0, ib_iters=10, cylinder=True):
    """Taylor-Green vortex with an artificial cylinder (Sec. 3.1.1).

    Box [-L, L]^2 with 2L + 1 nodes per side (node i at x = -L + i, the box
    edges are boundary nodes), tau = 0.65, Re = u0 L / nu = 10, a cylinder of
    diameter L at the centre whose markers move with the analytic velocity,
    the box's nodes held at the analytic velocity by non-equilibrium
    extrapolation.  The analytic solution is tgv_solution(); the run ends at
    t* = t u0 / L = 1, i.e. after L / u0 steps."""
    n = 2 * int(L) + 1
    nu = (tau - 0.5) / 3.0
    u0 = Re * nu / L
    c = float(L)  # lattice coordinate of the centre
    bodies = []
    if cylinder:
        R = L / 2.0
        nm = int(round(math.pi * L))
        xy = circle_markers(c, c, R, nm)
        bodies.append(dict(kind=FIXED, n=nm, xy=xy, uv=tgv_velocity_at(xy - c, 0.0, u0, L, nu),
                           ds=np.full(nm, 2 * math.pi * R / nm), xc=(c, c), U=(0.0, 0.0), omega=0.0,
                           theta=0.0, radius=R, rho_s=0.0))
    return dict(name="tgv_L%d" % L, nx=n, ny=n, tau=tau, rho0=1.0, bc=(DIRICHLET,) * 4, u_in=(0.0, 0.0),
                u_init=(0.0, 0.0), ib_iters=ib_iters, precision=precision, gravity=(0.0, 0.0), bodies=bodies,
                mrt_s=None, meta=dict(L=L, u0=u0, nu=nu, centre=c, steps=int(round(L / u0))))


def tgv_velocity_at(p, t, u0, L, nu):
    """Analytic TGV velocity (Eq. 30, with u_y of the sign that makes the
    field divergence-free) at points p[:, 2] measured from the box centre."""
    k = math.pi / L
    dec = math.exp(-2.0 * nu * k * k * t)
    x, y = p[:, 0], p[:, 1]
    return np.stack([-u0 * np.cos(k * x) * np.sin(k * y) * dec, u0 * np.sin(k * x) * np.cos(k * y) * dec], axis=1)


def tgv_solution(case, t):
    """(rho, u_x, u_y) of the analytic TGV on the case's nodes at time t:
    rho = rho0 - (3 u0^2 / 4)(cos 2kx + cos 2ky) exp(-4 nu k^2 t), the pressure
    of the Taylor-Green flow over c_s^2 = 1/3."""
    m = case["meta"]
    L, u0, nu, c = m["L"], m["u0"], m["nu"], m["centre"]
    n = case["nx"]
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    x -= c
    y -= c
    k = math.pi / L
    dec = math.exp(-2.0 * nu * k * k * t)
    ux = -u0 * np.cos(k * x) * np.sin(k * y) * dec
    uy = u0 * np.sin(k * x) * np.cos(k * y) * dec
    rho = case["rho0"] - 0.75 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y)) * dec * dec
    return rho, ux, uy


def tgv_boundary(case, t):
    """Analytic velocities of the perimeter nodes at time t."""
    m = case["meta"]
    p = perimeter_nodes(case["nx"], case["ny"]) - m["centre"]
    return tgv_velocity_at(p, t, m["u0"], m["L"], m["nu"])


def tgv_markers(case, t):
    """Analytic velocities of the cylinder's markers at time t."""
    m = case["meta"]
    b = case["bodies"][0]
    return tgv_velocity_at(b["xy"] - m["centre"], t, m["u0"], m["L"], m["nu"])


def batch(seed=0, count=256, precision=F32):
    """Uneven mix: each member is a Couette case (side uniform in 64..512) or a
    fixed cylinder in a 20D x 10D channel (D uniform in 16..64, Re uniform in
    10..100, U = 0.05, centre (5D, 5D))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        if rng.random() < 0.5:
            side = int(rng.integers(64, 513))
            out.append(couette(side=side, precision=precision))
        else:
            D = int(rng.integers(16, 65))
            Re = float(rng.uniform(10.0, 100.0))
            out.append(cylinder(nx=20 * D, ny=10 * D, D=float(D), centre=(5.0 * D, 5.0 * D),
                                U=0.05, Re=Re, precision=precision))
    return out


def arrivals(seed=0, rate=20.0, count=200, nx=400, ny=4000, steps=2000, precision=F32):
    """Poisson arrivals of settling requests: arrival time (s) and case."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    reqs = []
    for k in range(count):
        D = float(rng.uniform(16.0, 40.0))
        ratio = float(rng.uniform(1.01, 1.5))
        two = bool(rng.random() < 0.5)
        case = settling(nx=nx, ny=ny, D=D, density_ratio=ratio, two=two, precision=precision,
                        lower=(nx / 2.0, ny - 400.0))
        reqs.append(dict(t_arrive=float(t[k]), case=case, steps=steps, id=k))
    return reqs


def random_populations(seed, nx, ny, base, amp=0.02):
    """Positive populations base[i] * (1 + amp * noise), [9, ny, nx] float64.
    The caller supplies the nine base values (for example a rest state)."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64).reshape(9, 1, 1)
    return base * (1.0 + amp * rng.standard_normal((9, ny, nx)))


def random_fields(seed, nx, ny, rho0=1.0, amp_rho=0.01, amp_u=0.02):
    rng = np.random.default_rng(seed)
    rho = rho0 * (1.0 + amp_rho * rng.standard_normal((ny, nx)))
    ux = amp_u * rng.standard_normal((ny, nx))
    uy = amp_u * rng.standard_normal((ny, nx))
    return rho, ux, uy
