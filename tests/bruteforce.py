"""Independent numpy rewrites used to pin the oracle on tiny inputs.

Test code only.  Nothing here is shared with the oracle or the GPU library:
the lattice constants, the delta function and every rule below are written
again from the paper (Eqs. 1, 3, 4, 7, 15, 22-27) so that a mistake in either
implementation shows up as a disagreement.
"""
import numpy as np

# D2Q9, order fixed by the j_x and j_y rows of Eq. 5
E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
WTS = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
OPPOSITE = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def equilibrium(rho, ux, uy):
    """Eq. 3 on arrays; returns [9, ...]."""
    cu = E[:, 0].reshape((9,) + (1,) * np.ndim(rho)) * ux + E[:, 1].reshape(
        (9,) + (1,) * np.ndim(rho)) * uy
    w = WTS.reshape((9,) + (1,) * np.ndim(rho))
    return w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (ux ** 2 + uy ** 2))


def moments(f):
    rho = f.sum(axis=0)
    jx = np.tensordot(E[:, 0], f, axes=(0, 0))
    jy = np.tensordot(E[:, 1], f, axes=(0, 0))
    return rho, jx / rho, jy / rho


def bgk_periodic_step(f, tau):
    """One BGK collide + periodic stream with np.roll (f: [9, ny, nx])."""
    rho, ux, uy = moments(f)
    fp = f - (f - equilibrium(rho, ux, uy)) / tau
    out = np.empty_like(fp)
    for i in range(9):
        out[i] = np.roll(np.roll(fp[i], E[i, 1], axis=0), E[i, 0], axis=1)
    return out


def bgk_walled_step(f, tau):
    """One BGK collide + stream in a closed box with half-way bounce-back on all
    four sides: a population that would leave the box comes back reversed at the
    node it left (f: [9, ny, nx])."""
    rho, ux, uy = moments(f)
    fp = f - (f - equilibrium(rho, ux, uy)) / tau
    ny, nx = f.shape[1:]
    out = np.zeros_like(fp)
    for i in range(9):
        ex, ey = E[i]
        for y in range(ny):
            for x in range(nx):
                tx, ty = x + ex, y + ey
                if 0 <= tx < nx and 0 <= ty < ny:
                    out[i, ty, tx] += fp[i, y, x]
                else:
                    out[OPPOSITE[i], y, x] += fp[i, y, x]
    return out


def phi4(r):
    """4-point cosine kernel, Eq. 15(c)."""
    a = np.abs(r)
    return np.where(a <= 2.0, 0.25 * (1.0 + np.cos(np.pi * a / 2.0)), 0.0)


def interp_matrix(markers, nx, ny):
    """Dense P[l, y*nx + x] = D(x - X_l) on a periodic lattice (Eq. 15 with dx = 1)."""
    P = np.zeros((len(markers), nx * ny))
    xs = np.arange(nx)
    ys = np.arange(ny)
    for l, (X, Y) in enumerate(markers):
        # periodic images: shortest signed distance
        dx = (xs - X + nx / 2.0) % nx - nx / 2.0
        dy = (ys - Y + ny / 2.0) % ny - ny / 2.0
        P[l] = np.outer(phi4(dy), phi4(dx)).ravel()
    return P


def dense_sweeps(f, markers, U, ds, iters):
    """The N sweeps of Sec. 2.3 written as dense matrix products on a periodic
    lattice, literal route (Eqs. 22-27): interpolate f and f^neq, desired f from
    f^neq + f^eq(rho*, U), deviation, spread with D * ds, correct.
    Returns the corrected field and the total force on all markers (Eq. 29)."""
    nine, ny, nx = f.shape
    P = interp_matrix(markers, nx, ny)
    g = f.reshape(9, -1).copy()
    F = np.zeros(2)
    for _ in range(iters):
        rho, ux, uy = moments(g)
        feq = equilibrium(rho, ux, uy)
        fstar = g @ P.T                       # Eq. 22a, [9, M]
        fneqstar = (g - feq) @ P.T            # Eq. 22b
        rhostar = P @ rho
        eqb = equilibrium(rhostar, U[:, 0], U[:, 1])
        dev = fneqstar + eqb - fstar          # Eqs. 23-25
        F -= (E.T @ dev) @ ds                 # Eq. 29
        g = g + (dev * ds) @ P                # Eqs. 26-27
    return g.reshape(9, ny, nx), F


PERIODIC, WALL, FREESLIP, VELOCITY, OUTFLOW, PRESSURE, DIRICHLET = range(7)


def general_step(f, tau, bc, u_in=(0.0, 0.0), rho_out=1.0, ub=None):
    """One BGK step written in push form with explicit loops (tiny grids only).

    bc = (west, east, south, north).  Each post-collision population moves to
    x + e_i.  A population that leaves through a west/east side follows that
    side's rule (this includes corners); one that leaves only through the
    south/north side follows that side's rule:
      WALL      -> comes back at the node it left, reversed (half-way bounce-back);
      FREESLIP  -> mirrored in y, arrives at (x + e_x, y) (specular reflection);
      VELOCITY / OUTFLOW -> dropped; the open columns are rebuilt afterwards:
      OUTFLOW (east): the populations with e_x = -1 at column nx-1 copy column nx-2;
      VELOCITY (west, non-equilibrium extrapolation): every population of column 0
      becomes f^eq(rho(1), U_in) + f(1) - f^eq(rho(1), u(1));
      PRESSURE (east, non-equilibrium extrapolation): every population of column
      nx-1 becomes f^eq(rho_out, u(nx-2)) + f(nx-2) - f^eq(rho(nx-2), u(nx-2));
      DIRICHLET (all four sides): every population of boundary node b becomes
      f^eq(rho(n), ub[b]) + f(n) - f^eq(rho(n), u(n)), n = the nearest interior
      node (diagonal at corners); ub is a dict {(x, y): (u, v)}."""
    rho, ux, uy = moments(f)
    fp = f - (f - equilibrium(rho, ux, uy)) / tau
    ny, nx = f.shape[1:]
    out = np.full_like(fp, np.nan)
    west, east, south, north = bc
    mirror = {i: [k for k in range(9) if E[k, 0] == E[i, 0] and E[k, 1] == -E[i, 1]][0] for i in range(9)}
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                ex, ey = E[i]
                tx, ty = x + ex, y + ey
                if west == PERIODIC:
                    tx %= nx
                if south == PERIODIC:
                    ty %= ny
                inx, iny = 0 <= tx < nx, 0 <= ty < ny
                v = fp[i, y, x]
                if inx and iny:
                    out[i, ty, tx] = v
                elif not inx:
                    side = west if tx < 0 else east
                    if side == WALL:
                        out[OPPOSITE[i], y, x] = v
                else:
                    side = south if ty < 0 else north
                    if side == WALL:
                        out[OPPOSITE[i], y, x] = v
                    elif side == FREESLIP:
                        out[mirror[i], y, tx] = v
                    # DIRICHLET: dropped, the node is rebuilt below
    if east == OUTFLOW:
        for i in range(9):
            if E[i, 0] == -1:
                out[i, :, nx - 1] = out[i, :, nx - 2]
    if west == DIRICHLET:
        new = {}
        for (x, y), (bu, bv) in ub.items():
            xn, yn = min(max(x, 1), nx - 2), min(max(y, 1), ny - 2)
            fn = out[:, yn, xn]
            r, u, v = moments(fn)
            new[(x, y)] = equilibrium(r, bu, bv) + fn - equilibrium(r, u, v)
        for (x, y), val in new.items():
            out[:, y, x] = val
    if east == PRESSURE:
        r2, u2, v2 = moments(out[:, :, nx - 2])
        out[:, :, nx - 1] = (equilibrium(np.full_like(r2, rho_out), u2, v2)
                             + out[:, :, nx - 2] - equilibrium(r2, u2, v2))
    if west == VELOCITY:
        r1, u1, v1 = moments(out[:, :, 1])
        out[:, :, 0] = (equilibrium(r1, np.full_like(r1, u_in[0]), np.full_like(r1, u_in[1]))
                        + out[:, :, 1] - equilibrium(r1, u1, v1))
    assert not np.isnan(out).any(), "a population was left undefined"
    return out
