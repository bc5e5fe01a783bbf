"""Python binding of liblbmib.so (include/lbmib.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  The binding
raises if the library has not been built or cannot be loaded; there is no
fallback.  PyTorch is optional and only supplies device memory and streams.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmib.so")

OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_UNSTABLE, ERR_STATE = range(6)
F64, F32_SHIFTED = 0, 1
PERIODIC, WALL, FREESLIP, VELOCITY, OUTFLOW, PRESSURE, DIRICHLET = range(7)
FIXED, FREE = 0, 1
BGK, MRT = 0, 1
MAX_BODIES = 8

_NAMES = {0: "LBM_OK", 1: "LBM_ERR_INVALID", 2: "LBM_ERR_NOMEM", 3: "LBM_ERR_DEVICE",
          4: "LBM_ERR_UNSTABLE", 5: "LBM_ERR_STATE"}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_NAMES.get(code, code), msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("rho0", ctypes.c_double), ("precision", ctypes.c_int32),
                ("bc_west", ctypes.c_int32), ("bc_east", ctypes.c_int32),
                ("bc_south", ctypes.c_int32), ("bc_north", ctypes.c_int32),
                ("u_in", ctypes.c_double * 2), ("u_init", ctypes.c_double * 2),
                ("ib_iters", ctypes.c_int32), ("gravity", ctypes.c_double * 2),
                ("collision", ctypes.c_int32), ("mrt_s", ctypes.c_double * 9), ("delta", ctypes.c_int32)]


class Body(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("xc", ctypes.c_double * 2), ("U", ctypes.c_double * 2),
                ("omega", ctypes.c_double), ("theta", ctypes.c_double), ("radius", ctypes.c_double),
                ("rho_s", ctypes.c_double)]


# (name, restype, argtypes) of every entry point of include/lbmib.h
_P, _D, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_DP = ctypes.POINTER(ctypes.c_double)
_ST = ctypes.c_int
SIGNATURES = [
    ("lbm_create", _ST, [ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    ("lbm_destroy", None, [_P]),
    ("lbm_last_error", ctypes.c_char_p, [_P]),
    ("ib_set_markers", _ST, [_P, _I32, _I32, _DP, _DP, _DP, ctypes.POINTER(Body)]),
    ("lbm_set_boundary_velocity", _ST, [_P, _DP]),
    ("ib_set_marker_velocities", _ST, [_P, _I32, _DP]),
    ("lbm_step", _ST, [_P, _I32]),
    ("lbm_sync", _ST, [_P]),
    ("lbm_step_count", _I64, [_P]),
    ("ib_forces", _ST, [_P, _I32, _DP, _DP, _DP, ctypes.POINTER(Body)]),
    ("lbm_fields", _ST, [_P, _DP, _DP, _DP]),
    ("lbm_fields_device", _ST, [_P, _P, _P, _P]),
    ("lbm_fields_noalloc", _ST, [_P, _DP, _DP, _DP]),
    ("lbm_get_populations", _ST, [_P, _DP]),
    ("lbm_set_populations", _ST, [_P, _DP]),
    ("lbm_set_fields", _ST, [_P, _DP, _DP, _DP]),
    ("lbm_device_bytes", _SZ, [_P]),
    ("lbm_device_bytes_bound", _SZ, [ctypes.POINTER(Params), _I32, ctypes.POINTER(_I32)]),
    ("lbm_batch_create", _ST, [_I32, _SZ, _P, ctypes.POINTER(_P)]),
    ("lbm_batch_destroy", None, [_P]),
    ("lbm_batch_admit", _ST, [_P, _P, _I64]),
    ("lbm_batch_retire", _ST, [_P, _P]),
    ("lbm_batch_step", _ST, [_P, _I32]),
    ("lbm_batch_sync", _ST, [_P]),
    ("lbm_batch_remaining", _ST, [_P, _P, ctypes.POINTER(_I64)]),
    ("lbm_batch_bytes", _SZ, [_P]),
    ("lbm_batch_autotune", _ST, [_P, _I32, ctypes.POINTER(_I32)]),
    ("lbm_batch_set_tiling", _ST, [_P, _I32]),
    ("lbm_batch_get_tiling", _I32, [_P]),
    ("lbm_batch_set_lanes", _ST, [_P, _I32]),
    ("lbm_batch_get_lanes", _I32, [_P]),
    ("lbm_batch_get_lane_mode", _I32, [_P]),
    ("lbm_batch_lanes_concurrent", _I32, [_P]),
    ("lbm_tiling_count", _I32, []),
    ("lbm_tiling_info", _ST, [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("lbm_batch_profile", _ST, [_P, _I32, _DP, ctypes.POINTER(_I64)]),
    ("lbm_version", ctypes.c_char_p, []),
]

_lib = None


def load():
    """Load liblbmib.so; raises when it is missing (build it with build.py).

    When PyTorch is installed it is imported first: its HIP runtime then
    serves the library too (the library's libamdhip64.so.7 dependency resolves
    to the runtime torch already loaded), so device pointers and streams can be
    shared and the process holds one HIP runtime."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbmib.so is not built (%s); run paper_1803_09380_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = np.ascontiguousarray(np.broadcast_to(a, shape))
    return a


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):  # torch.cuda.Stream
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def make_params(nx, ny, tau, rho0=1.0, precision=F64, bc=(PERIODIC,) * 4, u_in=(0.0, 0.0), u_init=(0.0, 0.0),
                ib_iters=10, gravity=(0.0, 0.0), collision=BGK, mrt_s=None, delta=4):
    p = Params()
    p.nx, p.ny, p.tau, p.rho0, p.precision = nx, ny, tau, rho0, precision
    p.bc_west, p.bc_east, p.bc_south, p.bc_north = bc
    p.u_in[:] = u_in
    p.u_init[:] = u_init
    p.ib_iters = ib_iters
    p.gravity[:] = gravity
    p.collision = collision
    p.mrt_s[:] = mrt_s if mrt_s is not None else [1.0 / tau] * 9
    p.delta = delta
    return p


def _case_params(case, precision=None, collision=None, mrt_s=None, delta=None):
    if collision is None:
        mrt_s = case.get("mrt_s") if mrt_s is None else mrt_s
        collision = BGK if mrt_s is None else MRT
    return make_params(case["nx"], case["ny"], case["tau"], rho0=case["rho0"],
                       precision=case["precision"] if precision is None else precision, bc=case["bc"],
                       u_in=case["u_in"], u_init=case["u_init"], ib_iters=case["ib_iters"],
                       gravity=case["gravity"], collision=collision, mrt_s=mrt_s,
                       delta=case.get("delta", 4) if delta is None else delta)


def device_bytes_bound(case, precision=None):
    """lbm_device_bytes_bound for a workloads.py case: an upper bound on the
    device memory of Sim.from_case(case, precision), computed on the host
    without creating anything."""
    p = _case_params(case, precision)
    n = len(case["bodies"])
    counts = (_I32 * max(1, n))(*[int(b["n"]) for b in case["bodies"]])
    return int(load().lbm_device_bytes_bound(ctypes.byref(p), n, counts))


class Sim:
    """One simulation (lbm_sim)."""

    def __init__(self, nx, ny, tau, rho0=1.0, precision=F64, bc=(PERIODIC,) * 4, u_in=(0.0, 0.0),
                 u_init=(0.0, 0.0), ib_iters=10, gravity=(0.0, 0.0), stream=None, collision=BGK,
                 mrt_s=None, delta=4):
        L = load()
        p = make_params(nx, ny, tau, rho0=rho0, precision=precision, bc=bc, u_in=u_in, u_init=u_init,
                        ib_iters=ib_iters, gravity=gravity, collision=collision, mrt_s=mrt_s, delta=delta)
        h = _P()
        rc = L.lbm_create(ctypes.byref(p), _stream_handle(stream), ctypes.byref(h))
        if rc != OK:
            raise LbmError(rc, "lbm_create rejected the parameters")
        self._h = h
        self.nx, self.ny, self.precision = nx, ny, precision

    @classmethod
    def from_case(cls, case, precision=None, stream=None, collision=None, mrt_s=None, delta=None):
        """Create from a workloads.py case dict and set its bodies.  The
        collision follows the case's "mrt_s" and the delta function the
        case's "delta" (default 4) unless given."""
        if collision is None:
            mrt_s = case.get("mrt_s") if mrt_s is None else mrt_s
            collision = BGK if mrt_s is None else MRT
        s = cls(case["nx"], case["ny"], case["tau"], rho0=case["rho0"],
                precision=case["precision"] if precision is None else precision, bc=case["bc"],
                u_in=case["u_in"], u_init=case["u_init"], ib_iters=case["ib_iters"],
                gravity=case["gravity"], stream=stream, collision=collision, mrt_s=mrt_s,
                delta=case.get("delta", 4) if delta is None else delta)
        for k, b in enumerate(case["bodies"]):
            s.set_body(k, b["kind"], b["n"], xy=b["xy"], uv=b["uv"], ds=b["ds"], xc=b["xc"], U=b["U"],
                       omega=b["omega"], theta=b["theta"], radius=b["radius"], rho_s=b["rho_s"])
        return s

    def _check(self, rc, what):
        if rc != OK:
            msg = load().lbm_last_error(self._h)
            raise LbmError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_body(self, bid, kind, n, xy=None, uv=None, ds=None, xc=(0.0, 0.0), U=(0.0, 0.0), omega=0.0,
                 theta=0.0, radius=0.0, rho_s=0.0):
        b = Body()
        b.kind = kind
        b.xc[:] = xc
        b.U[:] = U
        b.omega, b.theta, b.radius, b.rho_s = omega, theta, radius, rho_s
        xy = _f64(xy)
        uv = _f64(uv)
        ds = _f64(ds)
        self._check(load().ib_set_markers(self._h, bid, n, _dp(xy), _dp(uv), _dp(ds), ctypes.byref(b)),
                    "ib_set_markers")

    def set_boundary_velocity(self, ub):
        """(u, v) of every perimeter node of a DIRICHLET box, shape (2 nx + 2 (ny - 2), 2)
        in the order south row, north row, west column, east column."""
        ub = _f64(ub)
        assert ub.size == 2 * (2 * self.nx + 2 * (self.ny - 2))
        self._check(load().lbm_set_boundary_velocity(self._h, _dp(ub)), "lbm_set_boundary_velocity")

    def set_marker_velocities(self, bid, uv):
        uv = _f64(uv)
        self._check(load().ib_set_marker_velocities(self._h, bid, _dp(uv)), "ib_set_marker_velocities")

    def step(self, n=1):
        self._check(load().lbm_step(self._h, n), "lbm_step")

    def sync(self):
        self._check(load().lbm_sync(self._h), "lbm_sync")

    @property
    def step_count(self):
        return load().lbm_step_count(self._h)

    def forces(self, bid):
        F, T, diag = np.zeros(2), np.zeros(1), np.zeros(2)
        st = Body()
        self._check(load().ib_forces(self._h, bid, _dp(F), _dp(T), _dp(diag), ctypes.byref(st)), "ib_forces")
        state = np.array([st.xc[0], st.xc[1], st.U[0], st.U[1], st.omega, st.theta])
        return F, float(T[0]), diag, state

    def fields(self):
        r, u, v = (np.empty((self.ny, self.nx)) for _ in range(3))
        self._check(load().lbm_fields(self._h, _dp(r), _dp(u), _dp(v)), "lbm_fields")
        return r, u, v

    def fields_noalloc(self):
        """fields() through the library's static staging array (no device allocation)."""
        r, u, v = (np.empty((self.ny, self.nx)) for _ in range(3))
        self._check(load().lbm_fields_noalloc(self._h, _dp(r), _dp(u), _dp(v)), "lbm_fields_noalloc")
        return r, u, v

    def fields_device(self, rho, ux, uy):
        """Write FP64 fields into device buffers (e.g. torch tensors' data_ptr())."""
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr() if hasattr(t, "data_ptr") else int(t))
        self._check(load().lbm_fields_device(self._h, ptr(rho), ptr(ux), ptr(uy)), "lbm_fields_device")

    def populations(self):
        f = np.empty((9, self.ny, self.nx))
        self._check(load().lbm_get_populations(self._h, _dp(f)), "lbm_get_populations")
        return f

    def set_populations(self, f):
        f = _f64(f)
        assert f.shape == (9, self.ny, self.nx)
        self._check(load().lbm_set_populations(self._h, _dp(f)), "lbm_set_populations")

    def set_fields(self, rho, ux, uy):
        shp = (self.ny, self.nx)
        r, u, v = _f64(rho, shp), _f64(ux, shp), _f64(uy, shp)
        self._check(load().lbm_set_fields(self._h, _dp(r), _dp(u), _dp(v)), "lbm_set_fields")

    @property
    def device_bytes(self):
        return load().lbm_device_bytes(self._h)


class Batch:
    """Many simulations of one precision stepped together (lbm_batch)."""

    def __init__(self, precision=F32_SHIFTED, hbm_budget=0, stream=None):
        h = _P()
        rc = load().lbm_batch_create(precision, hbm_budget, _stream_handle(stream), ctypes.byref(h))
        if rc != OK:
            raise LbmError(rc, "lbm_batch_create")
        self._h = h
        self.members = []

    def close(self):
        if getattr(self, "_h", None):
            load().lbm_batch_destroy(self._h)
            self._h = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, sim, steps=-1):
        """Returns True when admitted, False when over the HBM budget."""
        rc = load().lbm_batch_admit(self._h, sim.handle, steps)
        if rc == ERR_NOMEM:
            return False
        if rc != OK:
            raise LbmError(rc, "lbm_batch_admit")
        self.members.append(sim)
        return True

    def retire(self, sim):
        rc = load().lbm_batch_retire(self._h, sim.handle)
        if rc != OK:
            raise LbmError(rc, "lbm_batch_retire")
        self.members.remove(sim)

    def step(self, n=1):
        rc = load().lbm_batch_step(self._h, n)
        if rc != OK:
            raise LbmError(rc, "lbm_batch_step")

    def sync(self):
        rc = load().lbm_batch_sync(self._h)
        if rc != OK:
            raise LbmError(rc, "lbm_batch_sync")

    def remaining(self, sim):
        r = _I64()
        rc = load().lbm_batch_remaining(self._h, sim.handle, ctypes.byref(r))
        if rc != OK:
            raise LbmError(rc, "lbm_batch_remaining")
        return r.value

    @property
    def bytes(self):
        return load().lbm_batch_bytes(self._h)

    def autotune(self, trials=5):
        k = _I32()
        rc = load().lbm_batch_autotune(self._h, trials, ctypes.byref(k))
        if rc != OK:
            raise LbmError(rc, "lbm_batch_autotune")
        return k.value

    def profile(self, nsteps):
        """Per-kernel milliseconds (sweep, boundary, correction, bookkeeping)
        summed over nsteps steps, and the nodes one sweep launch updates."""
        ms = np.zeros(4)
        cells = _I64()
        rc = load().lbm_batch_profile(self._h, nsteps, _dp(ms), ctypes.byref(cells))
        if rc != OK:
            raise LbmError(rc, "lbm_batch_profile")
        return ms, cells.value

    def set_tiling(self, k):
        rc = load().lbm_batch_set_tiling(self._h, k)
        if rc != OK:
            raise LbmError(rc, "lbm_batch_set_tiling")

    @property
    def tiling(self):
        """Index of the sweep tiling in use."""
        return load().lbm_batch_get_tiling(self._h)

    def set_lanes(self, n):
        """0: automatic, 1: one lane, 2: two lanes replayed independently,
        3: two lanes interleaved step by step (2 and 3 need a heavy/light
        split of the members), 4: two interleaved halves of equal node count
        (at least two members)."""
        rc = load().lbm_batch_set_lanes(self._h, n)
        if rc != OK:
            raise LbmError(rc, "lbm_batch_set_lanes")

    @property
    def lanes(self):
        """Lanes (streams) the batch replays its steps on."""
        return load().lbm_batch_get_lanes(self._h)

    @property
    def lane_mode(self):
        """The lane request in force (0 .. 4, as set_lanes takes it)."""
        return load().lbm_batch_get_lane_mode(self._h)

    @property
    def lanes_concurrent(self):
        """1 when the second lane's stream runs beside the batch stream, 0 when
        not, -1 before a second lane has run."""
        return load().lbm_batch_lanes_concurrent(self._h)


def tilings():
    L = load()
    out = []
    for k in range(L.lbm_tiling_count()):
        a, b, c = _I32(), _I32(), _I32()
        L.lbm_tiling_info(k, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        out.append((a.value, b.value, c.value))
    return out


def version():
    return load().lbm_version().decode()
