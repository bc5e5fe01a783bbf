"""Flow diagnostics of the validation cases, computed on the host from what the
library returns (fields, body forces, body states).

  * the Couette closed form of Eq. 34, its torque, and the L2 norms (relative
    over the annulus, absolute along theta = pi/2 as in Eq. 35);
  * force coefficients C_d, C_l of Eq. 36;
  * recirculation length L_w behind a fixed cylinder: distance along the wake
    axis from the cylinder's rear point to where the streamwise velocity turns
    from reversed to forward (Sec. 3.2);
  * separation angle: polar angle, measured from the rear stagnation point,
    where the tangential velocity just outside the surface changes sign, i.e.
    where the reversed flow of the recirculation bubble meets the attached flow;
  * Strouhal number St = f D / U0 (Eq. 36) from the lift-coefficient history,
    with the lift amplitude and mean drag over whole shedding periods;
  * event times of a settling particle pair (drafting, kissing, tumbling) from
    the centre-to-centre distance history (Sec. 3.3.2).

These are post-processing of outputs; none of them is part of the time step.
"""
import math

import numpy as np


def couette_utheta(r, R1, R2, omega1):
    """Eq. 34 (outer cylinder at rest): u_theta = (R1^2 - R^2 r^2) omega1 /
    ((1 - R^2) r) with R = R1 / R2."""
    R = R1 / R2
    r = np.asarray(r, dtype=np.float64)
    return (R1 * R1 - R * R * r * r) * omega1 / ((1.0 - R * R) * r)


def couette_torque(mu, omega1, R1, R2):
    """Torque of the fluid on the inner cylinder of the steady flow of Eq. 34,
    T = -4 pi mu omega1 R1^2 R2^2 / (R2^2 - R1^2) per unit length."""
    return -4.0 * math.pi * mu * omega1 * R1 * R1 * R2 * R2 / (R2 * R2 - R1 * R1)


def couette_errors(ux, uy, centre, R1, R2, omega1):
    """(relative L2 velocity error over the nodes of the annulus R1 < r < R2,
    absolute L2 error of Eq. 35 on the profile theta = pi/2), against Eq. 34.
    The profile is the node column through the centre above it, where u_theta
    points along -x and u_r along y."""
    ny, nx = ux.shape
    cx, cy = centre
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx, dy = x - cx, y - cy
    rr = np.hypot(dx, dy)
    m = (rr > R1) & (rr < R2)
    ut = couette_utheta(rr[m], R1, R2, omega1)
    ua, va = -ut * dy[m] / rr[m], ut * dx[m] / rr[m]
    rel = math.sqrt(np.mean((ux[m] - ua) ** 2 + (uy[m] - va) ** 2) / np.mean(ua ** 2 + va ** 2))
    col = int(round(cx))
    ys = np.arange(ny, dtype=np.float64) - cy
    p = (ys > R1) & (ys < R2)
    utp = couette_utheta(ys[p], R1, R2, omega1)
    e35 = math.sqrt(np.mean((ux[p, col] + utp) ** 2 + uy[p, col] ** 2))
    return rel, e35


def observed_order(h, err):
    """Least-squares slope of log(err) against log(h)."""
    return float(np.polyfit(np.log(np.asarray(h, dtype=np.float64)), np.log(np.asarray(err, dtype=np.float64)), 1)[0])


def force_coefficients(F, U0, D, rho=1.0):
    """(C_d, C_l) of Eq. 36 from the force (F_x, F_y) on the body."""
    q = 0.5 * rho * U0 * U0 * D
    return F[0] / q, F[1] / q


def bilinear(a, x, y):
    """Bilinear interpolation of a (ny, nx) node array at lattice coordinates
    (x, y) (scalars or arrays), node (i, j) at x = i, y = j."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    i0 = np.clip(np.floor(x).astype(np.int64), 0, a.shape[1] - 2)
    j0 = np.clip(np.floor(y).astype(np.int64), 0, a.shape[0] - 2)
    tx, ty = x - i0, y - j0
    return ((1 - tx) * (1 - ty) * a[j0, i0] + tx * (1 - ty) * a[j0, i0 + 1] +
            (1 - tx) * ty * a[j0 + 1, i0] + tx * ty * a[j0 + 1, i0 + 1])


def recirculation_length(ux, xc, yc, R, search=None):
    """L_w: from the rear point (xc + R, yc) along the wake axis to the first
    point where u_x changes from negative to non-negative (linear between
    nodes; the axis row is interpolated when yc is not a node row).  Reversed
    flow must start within `search` lattice units behind the rear point
    (default R: the smeared interface may leave a thin layer of small positive
    u_x right at the surface); otherwise there is no bubble and 0 is returned."""
    nx = ux.shape[1]
    xs = np.arange(nx, dtype=np.float64)
    row = bilinear(ux, xs, np.full(nx, float(yc)))
    lim = xc + R + (R if search is None else search)
    k = int(math.floor(xc + R)) + 1
    while k < nx and row[k] >= 0:
        k += 1
        if xs[min(k, nx - 1)] > lim:
            return 0.0
    if k >= nx:
        return 0.0
    while k < nx and row[k] < 0:
        k += 1
    if k >= nx:
        return float("nan")
    x0, x1, u0, u1 = xs[k - 1], xs[k], row[k - 1], row[k]
    xz = x0 - u0 * (x1 - x0) / (u1 - u0)
    return xz - (xc + R)


def tangential_velocity(ux, uy, xc, yc, r, phi):
    """u_theta on the circle of radius r at polar angles phi (from +x, counter-clockwise)."""
    x = xc + r * np.cos(phi)
    y = yc + r * np.sin(phi)
    u = bilinear(ux, x, y)
    v = bilinear(uy, x, y)
    return -u * np.sin(phi) + v * np.cos(phi)


def separation_angles(ux, uy, xc, yc, R, offset=1.0, resolution_deg=0.05, front_skip_deg=10.0):
    """Separation angles (degrees from the rear stagnation point) of the upper
    and lower halves for a flow in +x, sampled on the circle r = R + offset.

    Along the attached boundary layer the flow runs from the front towards the
    rear (u_theta < 0 in the upper half); inside the recirculation bubble it
    runs the other way.  Scanning from the front (skipping the stagnation
    region) towards the rear, the angle is the first sign change, by linear
    interpolation between samples.  The lower half is scanned with the sign
    mirrored.  0 when the flow stays attached up to the rear point."""
    n = int(round(180.0 / resolution_deg)) + 1
    deg = np.linspace(180.0 - front_skip_deg, 0.0, n)
    out = []
    for sign in (1.0, -1.0):
        phi = sign * np.radians(deg)
        ut = sign * tangential_velocity(ux, uy, xc, yc, R + offset, phi)
        k = 0
        while k < n and ut[k] <= 0:
            k += 1
        if k >= n:
            out.append(0.0)
            continue
        if k == 0:
            out.append(float("nan"))
            continue
        d0, d1, a0, a1 = deg[k - 1], deg[k], ut[k - 1], ut[k]
        out.append(d0 - a0 * (d1 - d0) / (a1 - a0))
    return tuple(out)


def separation_angle_at_surface(ux, uy, xc, yc, R, offsets=(1.0, 1.5, 2.0, 2.5, 3.0), **kw):
    """Separation angle extrapolated to the surface: the angle found on
    circles r = R + h for the given offsets h (mean of both halves), fitted
    by a straight line in h and evaluated at h = 0.  Returns (angle, per-offset
    angles)."""
    vals = [float(np.mean(separation_angles(ux, uy, xc, yc, R, offset=h, **kw))) for h in offsets]
    a, b = np.polyfit(np.asarray(offsets, dtype=np.float64), np.asarray(vals), 1)
    return float(b), vals


def shedding(t, cl, cd=None, periods=None):
    """Strouhal analysis of a lift history sampled at times t (lattice steps).

    Upward crossings of the lift about its mean over the analysed window give
    the period (mean spacing of consecutive crossings, linear interpolation);
    with `periods` only the last that many whole periods are used.  Returns a
    dict with the period, frequency, lift amplitude (half the peak-to-peak over
    the whole periods) and the mean drag over the same periods (if cd is
    given), or None when fewer than two crossings are found."""
    t = np.asarray(t, dtype=np.float64)
    cl = np.asarray(cl, dtype=np.float64)
    m = cl.mean()
    s = cl - m
    idx = np.nonzero((s[:-1] < 0) & (s[1:] >= 0))[0]
    if len(idx) < 2:
        return None
    tc = t[idx] - s[idx] * (t[idx + 1] - t[idx]) / (s[idx + 1] - s[idx])
    if periods is not None and len(tc) > periods + 1:
        tc = tc[-(periods + 1):]
    T = float(np.mean(np.diff(tc)))
    win = (t >= tc[0]) & (t <= tc[-1])
    res = {"period": T, "frequency": 1.0 / T, "cycles": len(tc) - 1,
           "cl_amplitude": float(0.5 * (cl[win].max() - cl[win].min())),
           "cl_mean": float(cl[win].mean())}
    if cd is not None:
        res["cd_mean"] = float(np.asarray(cd, dtype=np.float64)[win].mean())
    return res


def strouhal(period, D, U0):
    """St = f D / U0 (Eq. 36) with f = 1/period (periods and U0 in lattice units)."""
    return D / (U0 * period)


def dkt_events(t, dist, D, contact_gap=None):
    """Events of a settling pair from the centre distance history dist(t):

      * drafting: the first time the distance has fallen 1% of its initial
        value below it (the gap starts to close);
      * kissing: the first local minimum of the distance that is within
        `contact_gap` (default D/4) of contact (distance D);
      * tumbling: the first time after kissing that the distance exceeds its
        value at kissing by D/4 (the pair separates).

    Returns a dict of the three times (None when an event does not occur)."""
    t = np.asarray(t, dtype=np.float64)
    d = np.asarray(dist, dtype=np.float64)
    gap = 0.25 * D if contact_gap is None else contact_gap
    ev = {"drafting": None, "kissing": None, "tumbling": None}
    below = np.nonzero(d < 0.99 * d[0])[0]
    if len(below):
        ev["drafting"] = float(t[below[0]])
    k_kiss = None
    for k in range(1, len(d) - 1):
        if d[k] <= d[k - 1] and d[k] <= d[k + 1] and d[k] < D + gap:
            k_kiss = k
            break
    if k_kiss is not None:
        ev["kissing"] = float(t[k_kiss])
        after = np.nonzero(d[k_kiss:] > d[k_kiss] + 0.25 * D)[0]
        if len(after):
            ev["tumbling"] = float(t[k_kiss + after[0]])
    return ev
