"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: closed
forms, exact identities, and independent numpy rewrites (tests/bruteforce.py).
"""
import math

import numpy as np
import pytest

import bruteforce as bf
from paper_1803_09380_amd import workloads as wl

REST = bf.WTS  # rest-state populations of the test's own lattice table


# ---------------------------------------------------------------- Eq. 15

@pytest.mark.parametrize("kind,support", [(2, 1), (3, 2), (4, 2)])
def test_delta_partition_of_unity(po, kind, support):
    rng = np.random.default_rng(1)
    for r in rng.random(2000):
        js = np.arange(-support - 1, support + 3)
        s = sum(po.delta(kind, j - r) for j in js)
        assert abs(s - 1.0) < 1e-14


def test_delta_cosine_even_odd_and_square(po):
    """Eq. 15(c): even and odd nodes each carry 1/2; sum of squares is 3/8."""
    rng = np.random.default_rng(2)
    for r in rng.random(2000):
        vals = {j: po.delta(4, j - r) for j in range(-3, 5)}
        even = sum(v for j, v in vals.items() if j % 2 == 0)
        odd = sum(v for j, v in vals.items() if j % 2 != 0)
        assert abs(even - 0.5) < 1e-14 and abs(odd - 0.5) < 1e-14
        assert abs(sum(v * v for v in vals.values()) - 3.0 / 8.0) < 1e-14


def test_delta_first_moment(po):
    """Eq. 15(a), (b) have a zero first moment.  The cosine kernel (c) does not:
    sum_j (j - r) phi(j - r) = (1 - 2r)/2 + (sin(pi r/2) - cos(pi r/2))/2."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for r in rng.random(2000):
        for kind in (2, 3):
            m = sum((j - r) * po.delta(kind, j - r) for j in range(-3, 5))
            assert abs(m) < 1e-14
        m4 = sum((j - r) * po.delta(4, j - r) for j in range(-3, 5))
        closed = (1 - 2 * r) / 2 + (math.sin(math.pi * r / 2) - math.cos(math.pi * r / 2)) / 2
        assert abs(m4 - closed) < 1e-14
        worst = max(worst, abs(m4))
    assert 0.02 < worst < 0.0212


def test_delta_values(po):
    assert po.delta(4, 0.0) == 0.5
    assert po.delta(4, 2.0) == 0.0 and po.delta(4, 2.5) == 0.0
    assert abs(po.delta(4, 1.0) - 0.25) < 1e-16
    assert abs(po.delta(3, 0.0) - 2.0 / 3.0) < 1e-16
    assert po.delta(2, 0.25) == 0.75


# ---------------------------------------------------------------- Eqs. 3-8

def test_equilibrium_moments(po):
    rng = np.random.default_rng(4)
    for _ in range(200):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(2)
        f = po.feq(rho, u[0], u[1])
        assert abs(f.sum() - rho) < 1e-14
        j = bf.E.T @ f
        assert np.allclose(j, rho * u, atol=1e-15, rtol=0)
        Pi = np.einsum("ia,ib,i->ab", bf.E, bf.E, f)
        assert np.allclose(Pi, rho * np.outer(u, u) + rho / 3 * np.eye(2), atol=1e-14, rtol=0)
        assert np.allclose(f, bf.equilibrium(np.array(rho), np.array(u[0]), np.array(u[1])),
                           atol=1e-15, rtol=0)


def test_mrt_matrix_inverse_and_bgk_limit(po):
    M, Minv = po.mrt_matrix()
    assert np.allclose(M @ Minv, np.eye(9), atol=1e-15)
    # rows j_x and j_y of Eq. 5 fix the velocity ordering of the lattice
    assert (M[3] == bf.E[:, 0]).all() and (M[5] == bf.E[:, 1]).all()
    rng = np.random.default_rng(5)
    tau = 0.73
    o_bgk = po.Oracle(8, 8, tau, collision=po.BGK)
    o_mrt = po.Oracle(8, 8, tau, collision=po.MRT, mrt_s=[1 / tau] * 9)
    paper = [1.0, 1.1, 1.25, 1.0, 1.8, 1.0, 1.8, 1 / tau, 1 / tau]  # rates of Sec. 3
    o_paper = po.Oracle(8, 8, tau, collision=po.MRT, mrt_s=paper)
    for _ in range(50):
        f = REST * (1 + 0.05 * rng.standard_normal(9))
        a, b = o_bgk.collide_node(f), o_mrt.collide_node(f)
        assert np.allclose(a, b, atol=1e-15, rtol=0)
        rho, ux, uy = bf.moments(f)
        ref = f - (f - bf.equilibrium(np.array(rho), np.array(ux), np.array(uy))) / tau
        assert np.allclose(a, ref, atol=1e-15, rtol=0)
        c = o_paper.collide_node(f)
        assert abs(c.sum() - f.sum()) < 1e-15
        assert np.allclose(bf.E.T @ c, bf.E.T @ f, atol=1e-15, rtol=0)


def _equilibrium_moments(rho, ux, uy):
    """Moments of Eq. 3 in the basis of Eq. 5, worked out by hand from the
    lattice sums sum w = 1, sum w e_a e_b = delta_ab / 3 and
    sum w e_a e_b e_c e_d = (delta_ab delta_cd + delta_ac delta_bd + delta_ad delta_bc) / 9:
    (rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy) =
    (rho, -2 rho + 3 rho |u|^2, rho - 3 rho |u|^2, rho u_x, -rho u_x, rho u_y,
    -rho u_y, rho (u_x^2 - u_y^2), rho u_x u_y)."""
    uu = ux * ux + uy * uy
    return np.array([rho, -2 * rho + 3 * rho * uu, rho - 3 * rho * uu, rho * ux, -rho * ux, rho * uy,
                     -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy])


def test_mrt_rows_give_the_equilibrium_moments(po):
    """Every row of the oracle's moment matrix (Eq. 5) maps the equilibrium of
    Eq. 3 onto its closed-form moment, the rows are mutually orthogonal with
    squared norms 9, 36, 36, 6, 12, 6, 12, 4, 4, and their entries are the
    integers of the printed matrix (a wrong sign or a swapped entry in any row
    breaks one of the three)."""
    M, _ = po.mrt_matrix()
    rng = np.random.default_rng(41)
    for _ in range(200):
        rho = 1 + 0.1 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(2)
        assert np.allclose(M @ po.feq(rho, u[0], u[1]), _equilibrium_moments(rho, u[0], u[1]),
                           atol=2e-15, rtol=0)
    G = M @ M.T
    assert np.array_equal(G, np.diag([9.0, 36, 36, 6, 12, 6, 12, 4, 4]))
    assert np.array_equal(M, np.round(M)) and np.abs(M).max() == 4


def test_mrt_relaxes_each_moment_at_its_own_rate(po):
    """Eq. 2 in moment space: m' = m - S (m - m^eq) with the diagonal S of
    Eq. 6, each moment at its own rate, m^eq from the closed form above (not
    from the oracle's equilibrium); the conserved moments keep their values."""
    M, _ = po.mrt_matrix()
    tau = 0.7
    rates = [1.0, 1.1, 1.25, 1.0, 1.8, 1.0, 1.8, 1 / tau, 1 / tau]
    o = po.Oracle(8, 8, tau, collision=po.MRT, mrt_s=rates)
    rng = np.random.default_rng(42)
    conserved = [0, 3, 5]
    for _ in range(100):
        f = REST * (1 + 0.08 * rng.standard_normal(9))
        m = M @ f
        meq = _equilibrium_moments(m[0], m[3] / m[0], m[5] / m[0])
        expect = m - np.array(rates) * (m - meq)
        expect[conserved] = m[conserved]
        assert np.allclose(M @ o.collide_node(f), expect, atol=2e-15, rtol=0)


# ---------------------------------------------------------------- Eq. 1 + boundary rules

def test_periodic_step_matches_numpy_roll(po):
    f = wl.random_populations(6, 11, 7, REST, amp=0.05)
    o = po.Oracle(11, 7, 0.77)
    o.set_populations(f)
    g = f.copy()
    for _ in range(3):
        o.step(1)
        g = bf.bgk_periodic_step(g, 0.77)
    assert np.allclose(o.populations(), g, atol=1e-15, rtol=0)


BC_CASES = [
    ("box_walls", (bf.WALL,) * 4),
    ("channel_inlet_outlet_freeslip", (bf.VELOCITY, bf.OUTFLOW, bf.FREESLIP, bf.FREESLIP)),
    ("periodic_x_walls_y", (bf.PERIODIC, bf.PERIODIC, bf.WALL, bf.WALL)),
    ("periodic_x_freeslip_y", (bf.PERIODIC, bf.PERIODIC, bf.FREESLIP, bf.FREESLIP)),
    ("wall_inlet_mix", (bf.VELOCITY, bf.WALL, bf.WALL, bf.FREESLIP)),
    ("wall_outlet_mix", (bf.WALL, bf.OUTFLOW, bf.FREESLIP, bf.WALL)),
    ("periodic_y_walls_x", (bf.WALL, bf.WALL, bf.PERIODIC, bf.PERIODIC)),
    ("channel_inlet_pressure_outlet", (bf.VELOCITY, bf.PRESSURE, bf.FREESLIP, bf.FREESLIP)),
    ("wall_pressure_mix", (bf.WALL, bf.PRESSURE, bf.WALL, bf.FREESLIP)),
    ("periodic_y_inlet_pressure", (bf.VELOCITY, bf.PRESSURE, bf.PERIODIC, bf.PERIODIC)),
]


@pytest.mark.parametrize("name,bc", BC_CASES, ids=[c[0] for c in BC_CASES])
def test_boundary_rules_match_push_bruteforce(po, name, bc):
    nx, ny = 7, 6
    f = wl.random_populations(7, nx, ny, REST, amp=0.05)
    u_in = (0.04, 0.01)
    o = po.Oracle(nx, ny, 0.81, bc=bc, u_in=u_in)
    o.set_populations(f)
    g = f.copy()
    for _ in range(3):
        o.step(1)
        g = bf.general_step(g, 0.81, bc, u_in)
    assert np.allclose(o.populations(), g, atol=1e-15, rtol=0)


def test_pressure_outlet_fixes_density_and_copies_velocity(po):
    """Non-equilibrium extrapolation at fixed density: the outlet column ends
    each step with density rho0 and the velocity of column nx-2, because the
    non-equilibrium parts carry no mass and no momentum."""
    nx, ny = 12, 9
    f = wl.random_populations(11, nx, ny, REST, amp=0.05)
    o = po.Oracle(nx, ny, 0.7, rho0=1.0, bc=(po.VELOCITY, po.PRESSURE, po.FREESLIP, po.FREESLIP), u_in=(0.03, 0.0))
    o.set_populations(f)
    for _ in range(4):
        o.step(1)
        rho, u, v = o.fields()
        assert np.allclose(rho[:, nx - 1], 1.0, atol=1e-14, rtol=0)
        assert np.allclose(u[:, nx - 1], u[:, nx - 2], atol=1e-15, rtol=0)
        assert np.allclose(v[:, nx - 1], v[:, nx - 2], atol=1e-15, rtol=0)


def test_pressure_outlet_needs_five_columns(po):
    with pytest.raises(Exception):
        po.Oracle(4, 6, 0.8, bc=(po.WALL, po.PRESSURE, po.WALL, po.WALL))


def test_prescribed_velocity_box_matches_push_bruteforce(po):
    nx, ny = 7, 6
    f = wl.random_populations(13, nx, ny, REST, amp=0.05)
    pts = wl.perimeter_nodes(nx, ny).astype(int)
    rng = np.random.default_rng(5)
    ubv = rng.normal(0, 0.03, size=(len(pts), 2))
    o = po.Oracle(nx, ny, 0.77, bc=(po.DIRICHLET,) * 4)
    o.set_populations(f)
    o.set_boundary_velocity(ubv)
    ub = {(int(x), int(y)): tuple(v) for (x, y), v in zip(pts, ubv)}
    g = f.copy()
    for _ in range(3):
        o.step(1)
        g = bf.general_step(g, 0.77, (bf.DIRICHLET,) * 4, ub=ub)
    assert np.allclose(o.populations(), g, atol=1e-15, rtol=0)
    # the boundary nodes carry the prescribed velocities exactly
    _, u, v = o.fields()
    assert np.allclose(u[pts[:, 1], pts[:, 0]], ubv[:, 0], atol=1e-15, rtol=0)
    assert np.allclose(v[pts[:, 1], pts[:, 0]], ubv[:, 1], atol=1e-15, rtol=0)


def _tgv_error(po, L, cylinder):
    from paper_1803_09380_amd import validate as val
    case = wl.tgv_cylinder(L, cylinder=cylinder)
    o = po.Oracle(case["nx"], case["ny"], case["tau"], bc=case["bc"])
    if cylinder:
        b = case["bodies"][0]
        o.set_body(0, po.FIXED, b["n"], xy=b["xy"], uv=b["uv"], ds=b["ds"])
    return val.tgv_run(o, case)["l2"]


@pytest.mark.parametrize("cylinder", [False, True])
def test_taylor_green_error_falls_at_third_order(po, cylinder):
    """Sec. 3.1.1: at fixed Re and tau, u0 = Re nu / L, so the absolute L2 error
    of Eq. 31 is u0 times a relative error; a second-order relative error makes
    the absolute one fall as L^-3.  Without the cylinder this checks the box
    boundary rule; with it, the paper's observation of nearly third order."""
    errs = [_tgv_error(po, L, cylinder=cylinder) for L in (8, 16, 32)]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(o > 2.7 for o in orders), (errs, orders)


def test_walled_box_conserves_mass(po):
    f = wl.random_populations(8, 20, 15, REST, amp=0.05)
    o = po.Oracle(20, 15, 0.9, bc=(po.WALL,) * 4)
    o.set_populations(f)
    m0 = f.sum()
    o.step(200)
    assert abs(o.populations().sum() - m0) < 1e-12 * m0


@pytest.mark.parametrize("outlet", ["outflow", "pressure"])
def test_uniform_channel_is_a_fixed_point(po, outlet):
    """Uniform flow at the inlet speed satisfies inlet, outlet and free-slip rules."""
    U = (0.05, 0.0)
    east = po.OUTFLOW if outlet == "outflow" else po.PRESSURE
    o = po.Oracle(24, 12, 0.62, bc=(po.VELOCITY, east, po.FREESLIP, po.FREESLIP), u_in=U,
                  u_init=U)
    o.step(50)
    r, u, v = o.fields()
    # a fixed point up to rounding (a wrong rule moves it by O(U^2) ~ 1e-3)
    assert np.abs(r - 1).max() < 1e-14 and np.abs(u - U[0]).max() < 1e-14 and np.abs(v).max() < 1e-14


# ---------------------------------------------------------------- Sec. 2.3 sweeps

def _rest_oracle(po, nx, ny, iters, route=None):
    kw = {} if route is None else dict(route=route)
    o = po.Oracle(nx, ny, 0.8, ib_iters=iters, **kw)
    return o


def test_single_marker_contraction_closed_form(po):
    """One marker on fluid at rest: the 16 stencil weights satisfy
    sum D^2 = (3/8)^2 = 9/64, so the momentum mismatch shrinks by exactly
    1 - 9 ds/64 per sweep and the force is -(64/9) dm0 (1 - q^N)."""
    for route in (po.LITERAL, po.SIMPLIFIED):
        N, ds = 10, 0.7
        U = np.array([0.01, -0.005])
        o = _rest_oracle(po, 16, 16, N, route)
        o.set_body(0, po.FIXED, 1, xy=np.array([[7.3, 8.6]]), uv=U[None, :], ds=np.array([ds]))
        o.ib_only()
        hist = o.residual_history()
        q = 1 - 9 * ds / 64
        expect = np.linalg.norm(U) * q ** np.arange(N)
        assert np.allclose(hist, expect, rtol=1e-12, atol=0)
        F, T, diag, _ = o.forces(0)
        assert np.allclose(F, -(64 / 9) * U * (1 - q ** N), rtol=1e-12, atol=0)
        assert abs(diag[0] - np.linalg.norm(U) * q ** N) < 1e-12 * np.linalg.norm(U)


def _arc(n, xc, yc, R, a0=0.3, step=0.09):
    a = a0 + step * np.arange(n)
    return np.stack([xc + R * np.cos(a), yc + R * np.sin(a)], axis=1)


def test_literal_route_equals_simplified_route(po):
    """Eq. 28 rewrites Eqs. 22-25; both must give the same corrected field."""
    f = wl.random_populations(9, 24, 20, REST, amp=0.03)
    xy = _arc(9, 12.0, 10.0, 6.0)
    uv = 0.01 * np.stack([np.cos(np.arange(9)), np.sin(np.arange(9))], axis=1)
    ds = np.full(9, 0.8)
    outs = []
    for route in (po.LITERAL, po.SIMPLIFIED):
        o = _rest_oracle(po, 24, 20, 10, route)
        o.set_populations(f)
        o.set_body(0, po.FIXED, 9, xy=xy, uv=uv, ds=ds, xc=(12.0, 10.0))
        o.ib_only()
        outs.append((o.populations(), o.forces(0)))
    assert np.abs(outs[0][0] - outs[1][0]).max() < 1e-15
    assert np.allclose(outs[0][1][0], outs[1][1][0], rtol=1e-12, atol=1e-17)


def test_sweeps_match_dense_bruteforce(po):
    """The oracle's sweeps equal a dense-matrix rewrite of Eqs. 22-27 on a tiny
    periodic lattice, with overlapping stencils and markers across the edge."""
    nx, ny = 14, 12
    f = wl.random_populations(10, nx, ny, REST, amp=0.03)
    xy = np.array([[3.2, 4.7], [4.1, 5.3], [5.05, 5.8], [12.9, 1.4], [0.6, 11.7]])
    uv = np.array([[0.01, 0.0], [0.008, 0.004], [0.0, 0.01], [-0.01, 0.002], [0.003, -0.007]])
    ds = np.array([1.0, 0.9, 1.1, 0.7, 1.3])
    o = _rest_oracle(po, nx, ny, 7, po.LITERAL)
    o.set_populations(f)
    o.set_body(0, po.FIXED, len(xy), xy=xy, uv=uv, ds=ds)
    o.ib_only()
    g, F = bf.dense_sweeps(f, xy, uv, ds, 7)
    assert np.abs(o.populations() - g).max() < 1e-15
    assert np.allclose(o.forces(0)[0], F, rtol=1e-12, atol=1e-18)


def test_sweeps_conserve_mass_and_balance_momentum(po):
    """Per node sum_i delta f_i = 0 (rho at the marker = interpolated rho), so the
    correction adds no mass; the body force of Eq. 29 is minus the momentum the
    corrections put into the fluid."""
    nx, ny = 30, 26
    f = wl.random_populations(11, nx, ny, REST, amp=0.03)
    o = _rest_oracle(po, nx, ny, 10)
    o.set_populations(f)
    xy1 = _arc(20, 15.0, 13.0, 7.0, step=0.15)
    xy2 = _arc(6, 15.0, 13.0, 2.5, a0=1.0, step=0.4)
    o.set_body(0, po.FIXED, 20, xy=xy1, ds=np.full(20, 1.0), xc=(15.0, 13.0))
    o.set_body(1, po.FIXED, 6, xy=xy2, ds=np.full(6, 1.0), xc=(15.0, 13.0), omega=0.004)
    m0 = f.sum()
    p0 = np.array([np.tensordot(bf.E[:, a], f, axes=(0, 0)).sum() for a in range(2)])
    o.ib_only()
    g = o.populations()
    p1 = np.array([np.tensordot(bf.E[:, a], g, axes=(0, 0)).sum() for a in range(2)])
    assert abs(g.sum() - m0) < 1e-13 * m0
    Ftot = o.forces(0)[0] + o.forces(1)[0]
    assert np.allclose(Ftot, -(p1 - p0), rtol=1e-10, atol=1e-16)


def test_couette_run_conserves_mass(po):
    c = wl.couette(32)
    o = po.Oracle(c["nx"], c["ny"], c["tau"], bc=c["bc"])
    for k, b in enumerate(c["bodies"]):
        o.set_body(k, b["kind"], b["n"], xy=b["xy"], ds=b["ds"], xc=b["xc"], omega=b["omega"])
    m0 = o.populations().sum()
    o.step(300)
    assert abs(o.populations().sum() - m0) < 1e-12 * m0


# ---------------------------------------------------------------- Eqs. 37-42 and 39

def test_collision_force_closed_form(po):
    R, gap, c, eps = 10.0, 1.0, 0.3, 0.01
    xi = np.array([0.0, 0.0])
    # touching: full strength c/eps along x_i - x_j
    F = po.collision_force(xi, [2 * R, 0.0], R, R, c, eps, gap)
    assert np.allclose(F, [-c / eps, 0.0], rtol=1e-14)
    # at the threshold gap and beyond: zero
    assert np.allclose(po.collision_force(xi, [0.0, 2 * R + gap], R, R, c, eps, gap), 0.0)
    assert np.allclose(po.collision_force(xi, [0.0, 2 * R + 2 * gap], R, R, c, eps, gap), 0.0)
    # half way: a quarter of the strength, along the diagonal
    d = 2 * R + 0.5 * gap
    F = po.collision_force(xi, [d / math.sqrt(2), d / math.sqrt(2)], R, R, c, eps, gap)
    assert np.allclose(F, -0.25 * c / eps * np.array([1, 1]) / math.sqrt(2), rtol=1e-13)


WALL_CASES = [  # side, bc tuple index, inward normal, gravity parallel to that side, side rule
    ("west", 0, (1.0, 0.0), (0.0, -1e-4), "wall"),
    ("east", 1, (-1.0, 0.0), (0.0, -1e-4), "wall"),
    ("south", 2, (0.0, 1.0), (1e-4, 0.0), "wall"),
    ("north", 3, (0.0, -1.0), (1e-4, 0.0), "wall"),
    ("south_freeslip", 2, (0.0, 1.0), (1e-4, 0.0), "freeslip"),
    ("north_freeslip", 3, (0.0, -1.0), (1e-4, 0.0), "freeslip"),
]


@pytest.mark.parametrize("side,idx,normal,g,rule", WALL_CASES, ids=[w[0] for w in WALL_CASES])
def test_wall_collision_acts_through_a_mirror_particle(po, side, idx, normal, g, rule):
    """Eq. 39 against a side: the wall sits half a spacing outside the first or
    last node row (half-way bounce-back, Fig. 2) and acts through a mirror
    particle of the same radius, so a circle whose surface is a gap h from the
    wall feels c/eps ((2h - xi)/xi)^2 along the inward normal while 2h < xi,
    c/eps at contact and nothing from h = xi/2 on (free-slip sides count as
    walls).  With no correction sweeps, no fluid velocity and gravity parallel
    to the wall, the first step's velocity change along the normal is that
    force over M_s (Eqs. 37, 41)."""
    nx, ny, R, rho_s = 40, 36, 5.0, 1.5
    gap, eps = 0.1 * R, 0.01
    V = math.pi * R * R
    Ms = rho_s * V
    c = (Ms - 1.0 * V) * math.hypot(*g)
    side_bc = po.WALL if rule == "wall" else po.FREESLIP
    bc = [po.PERIODIC] * 4
    if idx < 2:
        bc[0] = bc[1] = side_bc
    else:
        bc[2] = bc[3] = side_bc
    a = 0 if idx < 2 else 1
    lo, hi = -0.5, (nx if a == 0 else ny) - 0.5  # wall positions
    for h in (0.0, 0.1 * gap, 0.3 * gap, 0.5 * gap - 1e-9, 0.5 * gap, 0.6 * gap, 2.0):
        pos = [nx / 2.0, ny / 2.0]
        pos[a] = lo + R + h if idx in (0, 2) else hi - R - h
        o = po.Oracle(nx, ny, 0.8, bc=tuple(bc), ib_iters=0, gravity=g)
        o.set_body(0, po.FREE, 32, xc=pos, radius=R, rho_s=rho_s)
        o.step(1)
        _, _, _, st = o.forces(0)
        Fn = Ms * (st[2] * normal[0] + st[3] * normal[1])
        expect = c / eps * ((2 * h - gap) / gap) ** 2 if 2 * h < gap else 0.0
        assert abs(Fn - expect) <= 1e-12 * max(1.0, c / eps), (side, h, Fn, expect)


def test_no_wall_force_across_periodic_sides(po):
    """A circle next to a periodic seam feels no wall collision force."""
    R, rho_s = 5.0, 1.5
    o = po.Oracle(40, 36, 0.8, bc=(po.PERIODIC,) * 4, ib_iters=0, gravity=(0.0, -1e-4))
    o.set_body(0, po.FREE, 32, xc=(R - 0.5, 18.0), radius=R, rho_s=rho_s)
    o.step(1)
    assert o.forces(0)[3][2] == 0.0


def test_rigid_constant_force_is_a_parabola(po):
    """With no fluid (rho_f = 0) the update of Eqs. 41-42 is exact for a constant force."""
    R, rho_s = 5.0, 2.0
    M = rho_s * math.pi * R * R
    F = np.array([0.3, -0.7])
    st, prev = np.array([10.0, 20.0, 0.01, 0.02, 0.0, 0.0]), np.array([0.01, 0.02, 0.0])
    x0, u0 = st[:2].copy(), st[2:4].copy()
    for n in range(1, 41):
        st, prev = po.rigid_step(st, prev, F, 0.0, [0, 0], [0, 0], 0.0, rho_s, R)
        a = F / M
        assert np.allclose(st[:2], x0 + u0 * n + 0.5 * a * n * n, rtol=1e-13)
        assert np.allclose(st[2:4], u0 + a * n, rtol=1e-13)


def test_rigid_inertial_term_recursion(po):
    """No hydrodynamic or collision force: the lagged inertial term of Eq. 37
    gives a^n = (r a^{n-1}) - (1 - r) g, i.e. a^n = -g (1 - r^(n+1)), r = rho_f/rho_s."""
    R, rho_s, rho_f, g = 4.0, 1.25, 1.0, 1e-4
    r = rho_f / rho_s
    st, prev = np.zeros(6), np.zeros(3)
    for n in range(30):
        u_old = st[3]
        st, prev = po.rigid_step(st, prev, [0, 0], 0.0, [0, 0], [0, -g], rho_f, rho_s, R)
        a = st[3] - u_old
        assert abs(a - (-g * (1 - r ** (n + 1)))) < 1e-15


def test_rigid_rotation_update(po):
    """Torque only, no fluid: omega grows by T/I per step, theta by omega + T/(2I)."""
    R, rho_s = 3.0, 1.5
    I = 0.5 * rho_s * math.pi * R ** 4
    T = 2e-3
    st, prev = np.zeros(6), np.zeros(3)
    for n in range(1, 20):
        st, prev = po.rigid_step(st, prev, [0, 0], T, [0, 0], [0, 0], 0.0, rho_s, R)
        assert abs(st[4] - n * T / I) < 1e-15
        assert abs(st[5] - 0.5 * n * n * T / I) < 1e-14


def test_free_particle_sinks_and_markers_follow(po):
    """A free circle heavier than the fluid moves down; its markers stay on the circle."""
    c = wl.settling(nx=48, ny=96, D=10.0, density_ratio=1.5, lower=(24.0, 60.0))
    o = po.Oracle(c["nx"], c["ny"], c["tau"], bc=c["bc"], gravity=c["gravity"])
    b = c["bodies"][0]
    o.set_body(0, po.FREE, b["n"], xc=b["xc"], radius=b["radius"], rho_s=b["rho_s"])
    m0 = o.populations().sum()
    o.step(60)
    F, T, diag, st = o.forces(0)
    assert st[1] < 60.0 and st[3] < 0.0
    xy, uv, ds = o.body_markers(0, b["n"])
    rr = np.hypot(xy[:, 0] - st[0], xy[:, 1] - st[1])
    assert np.allclose(rr, b["radius"], rtol=1e-13)
    assert abs(o.populations().sum() - m0) < 1e-12 * m0


# ---------------------------------------------------------------- Couette, Eq. 34

def _couette_error(po, side, steps):
    """(relative L2 error over the annulus nodes, absolute L2 error of Eq. 35
    on the theta = pi/2 profile, inner torque, closed-form torque)."""
    c = wl.couette(side)
    m = c["meta"]
    o = po.Oracle(c["nx"], c["ny"], c["tau"], bc=c["bc"])
    for k, b in enumerate(c["bodies"]):
        o.set_body(k, b["kind"], b["n"], xy=b["xy"], ds=b["ds"], xc=b["xc"], omega=b["omega"])
    o.step(steps)
    r, u, v = o.fields()
    cx, cy = m["centre"]
    y, x = np.mgrid[0:side, 0:side]
    dx, dy = x - cx, y - cy
    rr = np.hypot(dx, dy)
    mask = (rr > m["R1"]) & (rr < m["R2"])
    ut = np.array([po.couette_utheta(q, m["R1"], m["R2"], m["omega1"]) for q in rr[mask]])
    ua, va = -ut * dy[mask] / rr[mask], ut * dx[mask] / rr[mask]
    err = math.sqrt(np.mean((u[mask] - ua) ** 2 + (v[mask] - va) ** 2) / np.mean(ua ** 2 + va ** 2))
    # Eq. 35: the profile theta = pi/2 (x = x_c, y > y_c), where u_theta points
    # along -x and u_r along y; absolute velocity error, no normalisation
    col = int(round(cx))
    ys = np.arange(side)
    prof = (ys - cy > m["R1"]) & (ys - cy < m["R2"])
    utp = np.array([po.couette_utheta(q, m["R1"], m["R2"], m["omega1"]) for q in (ys[prof] - cy)])
    err35 = math.sqrt(np.mean((u[prof, col] + utp) ** 2 + v[prof, col] ** 2))
    T = o.forces(1)[1]
    Ta = po.couette_torque_inner(m["nu"], m["omega1"], m["R1"], m["R2"])
    return err, err35, T, Ta


@pytest.mark.slow
def test_couette_profile_torque_and_order(po):
    """Eq. 34 closed form on the Couette geometry of the workloads (R1 = 12k,
    R2 = 24k, tau = 0.8, Re fixed), grids 32, 48, 64.  Refinement keeps tau and
    Re, so the wall speed scales as 1/k (diffusive scaling, as in Sec. 3.1.2).
    The L2 norm of Eq. 35 is an absolute velocity error: it falls at second
    order, the paper's observation; relative to the wall speed the error falls
    at first order (the same numbers divided by U).  The inner torque
    approaches -4 pi mu omega1 R1^2 R2^2 / (R2^2 - R1^2)."""
    res = {}
    for side in (32, 48, 64):
        k = side / 64.0
        res[side] = _couette_error(po, side, int(8000 * k * k))
    errs = [res[s][0] for s in (32, 48, 64)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.1
    rel_order = -np.polyfit(np.log([32, 48, 64]), np.log(errs), 1)[0]
    assert 0.85 < rel_order < 1.3, rel_order
    e35 = [res[s][1] for s in (32, 48, 64)]
    order35 = -np.polyfit(np.log([32, 48, 64]), np.log(e35), 1)[0]
    assert order35 > 1.8, (e35, order35)
    ratios = [res[s][2] / res[s][3] for s in (32, 48, 64)]
    assert all(r > 1.0 for r in ratios) and ratios[0] > ratios[1] > ratios[2]
    assert abs(ratios[2] - 1) < 0.15


@pytest.mark.slow
def test_paper_couette_set_up_is_first_order_relative_to_the_wall_speed(po):
    """Sec. 3.1.2's own set-up (MRT, Re = 10; here tau_s = 0.85, R = 0.5, outer
    radius on N = 20 and 40 spacings) against Eq. 34.  Refinement at fixed
    tau_s and Re halves the lattice wall speed, so the Eq. 35 norm in lattice
    units falls by about four while the error relative to the wall speed (and
    over the annulus) only halves: second order in lattice units, first order
    in the scale-free measure.  Forty sweeps instead of ten leave the errors
    within 0.5% (the slip left at the markers is not what limits them); the
    stored study (tests/golden/couette_paper_oracle.json, written by
    tests/couette_study.py) holds the same numbers."""
    import json
    import os
    import couette_study as cs
    e20 = cs.run_oracle(20, 0.5, 0.85)
    e40 = cs.run_oracle(40, 0.5, 0.85)
    lattice = math.log2(e20[0] / e40[0])
    relative = math.log2(e20[1] / e40[1])
    annulus = math.log2(e20[2] / e40[2])
    assert 1.8 < lattice < 2.2 and 0.8 < relative < 1.2 and 0.8 < annulus < 1.2, (lattice, relative, annulus)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "couette_paper_oracle.json")))
    ref = [s for s in gold["sets"] if (s["R"], s["tau_s"]) == (0.5, 0.85)][0]
    assert abs(e20[0] - ref["eq35_lattice"][0]) <= 1e-12 * e20[0]
    assert abs(e40[2] - ref["annulus_relative"][1]) <= 1e-12 * e40[2]
    case = wl.couette_paper(20, 0.5, 0.85, ib_iters=40)
    o = po.Oracle(case["nx"], case["ny"], case["tau"], bc=case["bc"], collision=po.MRT, mrt_s=case["mrt_s"],
                  ib_iters=40)
    for k, b in enumerate(case["bodies"]):
        o.set_body(k, b["kind"], b["n"], xy=b["xy"], ds=b["ds"], xc=b["xc"], omega=b["omega"])
    o.step(case["meta"]["steps"])
    _, ux, uy = o.fields()
    e20_40 = cs.errors(case, ux, uy)
    assert abs(e20_40[1] / e20[1] - 1) < 5e-3
