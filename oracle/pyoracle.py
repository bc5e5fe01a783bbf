"""ctypes view of the FP64 CPU oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle checks the GPU path; only the tests,
the smoke check and the CPU-baseline leg of the benchmark import this module.
It shares nothing with the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "lbm_oracle.c")

PERIODIC, WALL, FREESLIP, VELOCITY, OUTFLOW, PRESSURE, DIRICHLET = range(7)
BGK, MRT = 0, 1
LITERAL, SIMPLIFIED = 0, 1
FIXED, FREE = 0, 1
MAX_BODIES = 8


def build(force=False):
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP for the cell loops)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "lbm_oracle.h"))):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-Wall", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("tau", ctypes.c_double),
                ("rho0", ctypes.c_double), ("bc_west", ctypes.c_int), ("bc_east", ctypes.c_int),
                ("bc_south", ctypes.c_int), ("bc_north", ctypes.c_int),
                ("u_in", ctypes.c_double * 2), ("u_init", ctypes.c_double * 2),
                ("ib_iters", ctypes.c_int), ("delta", ctypes.c_int), ("route", ctypes.c_int),
                ("collision", ctypes.c_int), ("mrt_s", ctypes.c_double * 9),
                ("gravity", ctypes.c_double * 2)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_create.restype = P
        L.or_create.argtypes = [ctypes.POINTER(Params)]
        L.or_destroy.argtypes = [P]
        for name in ("or_set_populations", "or_get_populations"):
            getattr(L, name).argtypes = [P, dp]
        L.or_set_fields.argtypes = [P, dp, dp, dp]
        L.or_fields.argtypes = [P, dp, dp, dp]
        L.or_step_count.restype = ctypes.c_long
        L.or_step_count.argtypes = [P]
        L.or_set_body.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, D,
                                  D, D, D]
        L.or_body_markers.argtypes = [P, ctypes.c_int, dp, dp, dp]
        L.or_step.argtypes = [P, ctypes.c_int]
        L.or_set_boundary_velocity.argtypes = [P, dp]
        L.or_set_marker_velocities.argtypes = [P, ctypes.c_int, dp]
        L.or_ib_only.argtypes = [P]
        L.or_forces.argtypes = [P, ctypes.c_int, dp, dp, dp, dp]
        L.or_residual_history.argtypes = [P, dp, ctypes.c_int]
        L.or_delta.restype = D
        L.or_delta.argtypes = [ctypes.c_int, D]
        L.or_feq.argtypes = [D, D, D, dp]
        L.or_collide_node.argtypes = [P, dp, dp]
        L.or_mrt_matrix.argtypes = [dp, dp]
        L.or_couette_utheta.restype = D
        L.or_couette_utheta.argtypes = [D, D, D, D]
        L.or_couette_torque_inner.restype = D
        L.or_couette_torque_inner.argtypes = [D, D, D, D]
        L.or_collision_force.argtypes = [dp, dp, D, D, D, D, D, dp]
        L.or_rigid_step.argtypes = [dp, dp, dp, D, dp, dp, D, D, D]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One oracle simulation.  Arrays are numpy float64; fields are [ny, nx],
    populations [9, ny, nx]."""

    def __init__(self, nx, ny, tau, rho0=1.0, bc=(PERIODIC,) * 4, u_in=(0.0, 0.0),
                 u_init=(0.0, 0.0), ib_iters=10, delta=4, route=SIMPLIFIED, collision=BGK,
                 mrt_s=None, gravity=(0.0, 0.0)):
        p = Params()
        p.nx, p.ny, p.tau, p.rho0 = nx, ny, tau, rho0
        p.bc_west, p.bc_east, p.bc_south, p.bc_north = bc
        p.u_in[:] = u_in
        p.u_init[:] = u_init
        p.ib_iters, p.delta, p.route, p.collision = ib_iters, delta, route, collision
        p.mrt_s[:] = mrt_s if mrt_s is not None else [1.0 / tau] * 9
        p.gravity[:] = gravity
        self.nx, self.ny = nx, ny
        self.params = p
        self._h = lib().or_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def set_populations(self, f):
        f = _f64(f)
        assert f.shape == (9, self.ny, self.nx)
        lib().or_set_populations(self._h, _p(f))

    def populations(self):
        f = np.empty((9, self.ny, self.nx))
        lib().or_get_populations(self._h, _p(f))
        return f

    def set_fields(self, rho, ux, uy):
        r, u, v = (_f64(np.broadcast_to(a, (self.ny, self.nx))) for a in (rho, ux, uy))
        lib().or_set_fields(self._h, _p(r), _p(u), _p(v))

    def fields(self):
        r, u, v = (np.empty((self.ny, self.nx)) for _ in range(3))
        lib().or_fields(self._h, _p(r), _p(u), _p(v))
        return r, u, v

    @property
    def step_count(self):
        return lib().or_step_count(self._h)

    def set_body(self, bid, kind, n, xy=None, uv=None, ds=None, xc=(0.0, 0.0), U=(0.0, 0.0),
                 omega=0.0, theta=0.0, radius=0.0, rho_s=0.0):
        xy, uv, ds = _f64(xy), _f64(uv), _f64(ds)
        xc, U = _f64(xc), _f64(U)
        rc = lib().or_set_body(self._h, bid, kind, n, _p(xy), _p(uv), _p(ds), _p(xc), _p(U), omega,
                               theta, radius, rho_s)
        if rc:
            raise ValueError("oracle rejected body %d" % bid)

    def body_markers(self, bid, n):
        xy, uv, ds = np.empty((n, 2)), np.empty((n, 2)), np.empty(n)
        lib().or_body_markers(self._h, bid, _p(xy), _p(uv), _p(ds))
        return xy, uv, ds

    def set_boundary_velocity(self, ub):
        """ub[k] = (u, v) of perimeter node k (south row, north row, west
        column, east column; see lbm_oracle.h)."""
        ub = _f64(ub)
        if lib().or_set_boundary_velocity(self._h, _p(ub)) != 0:
            raise ValueError("not a prescribed-velocity box")

    def set_marker_velocities(self, bid, uv):
        uv = _f64(uv)
        if lib().or_set_marker_velocities(self._h, bid, _p(uv)) != 0:
            raise ValueError("not a fixed body")

    def step(self, n=1):
        lib().or_step(self._h, n)

    def ib_only(self):
        lib().or_ib_only(self._h)

    def forces(self, bid):
        F, T, diag, st = np.zeros(2), np.zeros(1), np.zeros(2), np.zeros(6)
        if lib().or_forces(self._h, bid, _p(F), _p(T), _p(diag), _p(st)):
            raise ValueError("no body %d" % bid)
        return F, float(T[0]), diag, st

    def residual_history(self):
        out = np.zeros(256)
        n = lib().or_residual_history(self._h, _p(out), 256)
        return out[:n].copy()

    def collide_node(self, f9):
        f9 = _f64(f9)
        out = np.empty(9)
        lib().or_collide_node(self._h, _p(f9), _p(out))
        return out


def delta(kind, r):
    return lib().or_delta(kind, float(r))


def feq(rho, ux, uy):
    out = np.empty(9)
    lib().or_feq(rho, ux, uy, _p(out))
    return out


def mrt_matrix():
    M, Minv = np.empty(81), np.empty(81)
    lib().or_mrt_matrix(_p(M), _p(Minv))
    return M.reshape(9, 9), Minv.reshape(9, 9)


def couette_utheta(r, R1, R2, omega1):
    return lib().or_couette_utheta(r, R1, R2, omega1)


def couette_torque_inner(mu, omega1, R1, R2):
    return lib().or_couette_torque_inner(mu, omega1, R1, R2)


def collision_force(xi, xj, Ri, Rj, cij, eps, gap):
    out = np.empty(2)
    lib().or_collision_force(_p(_f64(xi)), _p(_f64(xj)), Ri, Rj, cij, eps, gap, _p(out))
    return out


def rigid_step(st, prev, Fs, Ts, Fc, g, rho_f, rho_s, R):
    st = _f64(st).copy()
    prev = _f64(prev).copy()
    lib().or_rigid_step(_p(st), _p(prev), _p(_f64(Fs)), Ts, _p(_f64(Fc)), _p(_f64(g)), rho_f,
                        rho_s, R)
    return st, prev
