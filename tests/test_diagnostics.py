"""CPU pins of the host-side diagnostics on fields and histories whose answers
are known in closed form (bilinear interpolation is exact on linear fields)."""
import math

import numpy as np
import pytest

from paper_1803_09380_amd import diagnostics as dg


def test_force_coefficients_eq36():
    cd, cl = dg.force_coefficients(np.array([0.02, -0.005]), U0=0.1, D=40.0)
    assert cd == pytest.approx(0.02 / (0.5 * 0.01 * 40.0))
    assert cl == pytest.approx(-0.005 / (0.5 * 0.01 * 40.0))


def test_bilinear_is_exact_on_linear_fields():
    ny, nx = 30, 40
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    a = 0.3 * x - 1.7 * y + 2.0
    rng = np.random.default_rng(0)
    px, py = rng.uniform(0, nx - 1, 100), rng.uniform(0, ny - 1, 100)
    assert np.allclose(dg.bilinear(a, px, py), 0.3 * px - 1.7 * py + 2.0, atol=1e-12)


@pytest.mark.parametrize("yc", [20.0, 20.5, 20.25])
def test_recirculation_length_of_a_known_crossing(yc):
    """u_x = (x - xr)(x - xz) behind the body: reversed between the rear point
    xr and xz; made linear between nodes so the crossing is exact."""
    nx, ny = 120, 41
    xc, R = 30.0, 8.0
    xr, xz = xc + R, 61.0  # crossing on a node
    x = np.arange(nx, dtype=np.float64)
    row = np.where(x <= xr, 0.0, np.where(x < xz, -(x - xr) * 0.01, (x - xz) * 0.02))
    ux = np.tile(row, (ny, 1))
    assert dg.recirculation_length(ux, xc, yc, R) == pytest.approx(xz - xr, abs=1e-12)
    # crossing between nodes: linear interpolation of the two neighbours
    row2 = row.copy()
    row2[61] = 0.03  # u(60) = -0.22, u(61) = 0.03 -> zero at 60 + 0.22/0.25
    ux2 = np.tile(row2, (ny, 1))
    assert dg.recirculation_length(ux2, xc, yc, R) == pytest.approx(60.0 + 0.22 / 0.25 - xr, abs=1e-12)


def test_no_reversed_flow_gives_zero_length():
    ux = np.full((20, 60), 0.05)
    assert dg.recirculation_length(ux, 20.0, 10.0, 5.0) == 0.0


def _uniform_plus_rotation(U, w, xc, yc, nx, ny):
    """Uniform flow U in front of the body (x < xc); behind it (x >= xc)
    u = U - w |y - yc|, v = w (x - xc) sign(y - yc): the upper half of the
    rear turns with rate w and the lower half is its mirror image.  On a
    circle of radius r the tangential velocity in the upper half is then
    -U sin(phi) in front and w r - U sin(phi) behind, which changes sign at
    phi = asin(w r / U).  The kink sits on a node column, so bilinear
    interpolation reproduces the field exactly away from that column."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    rear = x >= xc
    ux = np.where(rear, U - w * np.abs(y - yc), U)
    uy = np.where(rear, w * (x - xc) * np.sign(y - yc), 0.0)
    return ux, uy


@pytest.mark.parametrize("w", [0.002, 0.004])
def test_separation_angle_closed_form(w):
    nx, ny, xc, yc, R = 101, 101, 50.0, 50.0, 12.0
    U, off = 0.1, 1.0
    ux, uy = _uniform_plus_rotation(U, w, xc, yc, nx, ny)
    up, lo = dg.separation_angles(ux, uy, xc, yc, R, offset=off, resolution_deg=0.01)
    exact = math.degrees(math.asin(w * (R + off) / U))
    # linear interpolation of a sine between samples 0.01 degrees apart
    assert up == pytest.approx(exact, abs=1e-4)
    assert lo == pytest.approx(exact, abs=1e-4)


def test_surface_extrapolation_of_a_linear_dependence():
    """With u_theta = w r - U sin(phi), sin(phi_sep) = w r / U grows linearly
    in r for small angles; with a field whose separation angle is exactly
    linear in the offset the extrapolation is exact."""
    nx, ny, xc, yc, R = 101, 101, 50.0, 50.0, 12.0
    U, w = 0.1, 0.002
    ux, uy = _uniform_plus_rotation(U, w, xc, yc, nx, ny)
    th, vals = dg.separation_angle_at_surface(ux, uy, xc, yc, R, offsets=(1.0, 2.0, 3.0), resolution_deg=0.01)
    exact = [math.degrees(math.asin(w * (R + h) / U)) for h in (1.0, 2.0, 3.0)]
    assert np.allclose(vals, exact, atol=1e-4)
    # the fitted line through nearly collinear points, evaluated at h = 0
    a, b = np.polyfit([1.0, 2.0, 3.0], exact, 1)
    assert th == pytest.approx(b, abs=1e-3)
    assert th == pytest.approx(math.degrees(math.asin(w * R / U)), abs=0.02)


def test_reversed_flow_behind_a_thin_positive_layer():
    """A layer of small positive u_x right behind the surface (smeared
    interface) does not hide the bubble that follows it."""
    nx, ny = 200, 41
    xc, R = 40.0, 10.0
    x = np.arange(nx, dtype=np.float64)
    row = np.where(x <= xc + R, 0.0, 0.0)
    row = np.where((x > xc + R) & (x < xc + R + 3), 1e-4, row)
    row = np.where((x >= xc + R + 3) & (x < 90.0), -0.01, row)
    row = np.where(x >= 90.0, 0.02 * (x - 89.5), row)
    ux = np.tile(row, (ny, 1))
    # u(89) = -0.01, u(90) = 0.01: zero at 89.5
    assert dg.recirculation_length(ux, xc, 20.0, R) == pytest.approx(89.5 - (xc + R), abs=1e-9)


def test_attached_flow_has_no_separation():
    ux, uy = _uniform_plus_rotation(0.1, 0.0, 50.0, 50.0, 101, 101)
    uy[:] = 0.0
    assert dg.separation_angles(ux, uy, 50.0, 50.0, 10.0) == (0.0, 0.0)


def test_shedding_frequency_amplitude_and_mean_drag():
    T = 2417.3
    t = np.arange(0, 30000, 10.0)
    cl = 0.35 * np.sin(2 * math.pi * t / T + 0.4) + 0.01
    cd = 1.4 + 0.01 * np.sin(4 * math.pi * t / T)
    res = dg.shedding(t, cl, cd, periods=8)
    assert res["period"] == pytest.approx(T, rel=1e-4)
    assert res["cycles"] == 8
    assert res["cl_amplitude"] == pytest.approx(0.35, rel=1e-3)
    assert res["cd_mean"] == pytest.approx(1.4, abs=2e-4)
    assert dg.strouhal(res["period"], D=40.0, U0=0.1) == pytest.approx(40.0 / (0.1 * T), rel=1e-4)


def test_steady_lift_has_no_period():
    assert dg.shedding(np.arange(100.0), np.full(100, 0.2)) is None


def test_dkt_events_of_a_piecewise_history():
    """Distance 40 until t=500, closing linearly to 21 at t=1300, flat (kissing)
    until 2500, then opening; drafting/kissing/tumbling read off exactly."""
    D = 20.0
    t = np.arange(0.0, 3500.0, 1.0)
    d = np.where(t < 500, 40.0, 40.0 - (t - 500) * 19.0 / 800.0)
    d = np.where(t >= 1300, 21.0 + 1e-6 * (t - 1300), d)
    d = np.where(t >= 2500, 21.0 + 1e-6 * 1200 + (t - 2500) * 0.05, d)
    ev = dg.dkt_events(t, d, D)
    # 1% below 40 is reached 0.4 / (19/800) after t = 500
    assert ev["drafting"] == pytest.approx(500 + math.ceil(0.4 * 800 / 19.0 + 1e-9), abs=1.0)
    assert ev["kissing"] == 1300.0
    assert ev["tumbling"] == pytest.approx(2500 + 5.0 / 0.05, abs=1.5)


def test_validation_reference_values_match_the_golden_files():
    """The paper's numbers used by the validation runner are the ones stored
    (with their citation) under tests/golden/."""
    import os
    from paper_1803_09380_amd import validate as val
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    present = {}
    for ln in open(os.path.join(gold, "table1_cylinder.txt")):
        f = ln.split()
        if f and not f[0].startswith("#") and f[0] == "present":
            present.setdefault(int(f[1]), {})[f[2]] = float(f[3])
    assert present == val.TABLE1_PAPER
    dkt = {}
    for ln in open(os.path.join(gold, "dkt_events.txt")):
        f = ln.split()
        if f and not f[0].startswith("#"):
            dkt[f[0]] = float(f[1])
    assert dkt == val.DKT_PAPER


def test_couette_closed_form_solves_the_ode_and_boundary_values():
    """Eq. 34 satisfies Eq. 32 (finite differences) and Eq. 33."""
    R1, R2, w = 12.0, 24.0, 0.01 / 12.0
    assert dg.couette_utheta(R1, R1, R2, w) == pytest.approx(w * R1, rel=1e-14)
    assert abs(dg.couette_utheta(R2, R1, R2, w)) < 1e-17
    r = np.linspace(13.0, 23.0, 11)
    h = 1e-3
    u = lambda q: dg.couette_utheta(q, R1, R2, w)
    d2 = (u(r + h) - 2 * u(r) + u(r - h)) / h ** 2
    dq = (u(r + h) / (r + h) - u(r - h) / (r - h)) / (2 * h)
    # the terms are about w / r ~ 1e-4; a wrong sign or power leaves residuals of that size
    assert np.abs(d2 + dq).max() < 1e-8


def test_couette_errors_vanish_on_the_exact_field():
    n, c, R1, R2, w = 65, (32.0, 32.0), 12.0, 24.0, 0.001
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    dx, dy = x - c[0], y - c[1]
    r = np.maximum(np.hypot(dx, dy), 1e-9)
    ut = dg.couette_utheta(r, R1, R2, w)
    ux, uy = -ut * dy / r, ut * dx / r
    rel, e35 = dg.couette_errors(ux, uy, c, R1, R2, w)
    assert rel < 1e-14 and e35 < 1e-17
    rel2, e352 = dg.couette_errors(1.01 * ux, 1.01 * uy, c, R1, R2, w)
    assert rel2 == pytest.approx(0.01, rel=1e-9)


def test_observed_order():
    h = np.array([1.0, 0.5, 0.25])
    assert dg.observed_order(h, 3.0 * h ** 2) == pytest.approx(2.0, abs=1e-12)
