"""ctypes wrapper of the FP64 CPU oracle (oracle/lbm_oracle.c).

TEST INFRASTRUCTURE ONLY (tests, the smoke check, the benchmark's CPU
baseline).  Arrays are numpy float64 / uint8 / int32 in the layout
[component][z][y][x] with x fastest; populations are [19][z][y][x] in the
oracle's own velocity order (see ``lattice()``).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)
_i64p = C.POINTER(C.c_int64)


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("z_periodic", C.c_int), ("srt", C.c_int),
                ("tau", C.c_double), ("magic", C.c_double), ("rho0", C.c_double),
                ("wall_u", C.c_double), ("g", C.c_double * 3), ("init_couette", C.c_int),
                ("coupling", C.c_int), ("stabilize", C.c_int),
                ("contact_k", C.c_double), ("contact_range", C.c_double),
                ("x_walls", C.c_int), ("y_walls", C.c_int), ("z_free_slip", C.c_int)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.or_lattice.argtypes = [_ip, _dp, _ip]
        L.or_feq.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.or_omega_odd.argtypes = [C.c_double, C.c_double, C.c_int]
        L.or_omega_odd.restype = C.c_double
        L.or_collide_cell.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.or_collide_cell_shift.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_segment_closest.argtypes = [_dp, _dp, C.c_double, _dp, _dp, C.c_double, _dp, _dp]
        L.or_segment_closest.restype = C.c_double
        L.or_contact_pair.argtypes = [_dp, C.c_double, C.c_double, _dp, _dp, C.c_double, C.c_double,
                                      C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.or_contact_pair.restype = C.c_double
        L.or_mean_velocity.argtypes = [C.c_void_p, _dp]
        L.or_mean_velocity.restype = C.c_int64
        L.or_fiber_axis.argtypes = [_dp, _dp]
        L.or_cell_inside.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double,
                                     C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_map.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp,
                             _ip, _i64p]
        L.or_body_inertia.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp]
        L.or_cell_inside_shape.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_int,
                                           C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_map_shapes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp,
                                    _dp, _ip, _ip, _i64p]
        L.or_rigid_step.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                    C.c_int, C.c_int, C.c_int, C.c_int, _dp]
        L.or_rigid_step_implicit.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp,
                                             _dp, _dp, _dp, _dp, C.c_int, C.c_int, C.c_int,
                                             C.c_int, _dp, _dp, _dp]
        L.or_create.argtypes = [C.POINTER(Params)]
        L.or_create.restype = C.c_void_p
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_add_fiber.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                   _dp, _dp]
        L.or_add_fiber_ex.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                      _dp, _dp, C.c_int, _dp, _dp]
        L.or_set_kinematics.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int64]
        L.or_set_correction.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.or_step.argtypes = [C.c_void_p, C.c_int64]
        L.or_get_populations.argtypes = [C.c_void_p, _dp]
        L.or_set_populations.argtypes = [C.c_void_p, _dp]
        L.or_get_fields.argtypes = [C.c_void_p, _dp, _dp, _u8p, _ip]
        L.or_get_fiber_state.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.or_get_force_torque.argtypes = [C.c_void_p, _dp, _dp]
        L.or_get_history.argtypes = [C.c_void_p, C.c_int64, C.c_int64, _dp]
        L.or_get_history.restype = C.c_int64
        L.or_overlaps.argtypes = [C.c_void_p]
        L.or_overlaps.restype = C.c_int64
        L.or_steps_done.argtypes = [C.c_void_p]
        L.or_steps_done.restype = C.c_int64
        L.or_nfibers.argtypes = [C.c_void_p]
        L.or_get_exchange_sums.argtypes = [C.c_void_p, _dp]
        L.or_set_mutation.argtypes = [C.c_int]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        _LIB = L
    return _LIB


def _d(a):
    return a.ctypes.data_as(_dp)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


# ---------------------------------------------------------------- building blocks
def lattice():
    c = np.zeros(57, np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    lib().or_lattice(c.ctypes.data_as(_ip), _d(w), opp.ctypes.data_as(_ip))
    return c.reshape(19, 3), w, opp


def feq(rho, rho0, u):
    out = np.zeros(19)
    lib().or_feq(rho, rho0, _d(_arr(u, 3)), _d(out))
    return out


def omega_odd(tau, magic, srt=False):
    return lib().or_omega_odd(tau, magic, int(srt))


def collide_cell(f, rho0, omega_e, omega_o, g=(0.0, 0.0, 0.0)):
    out = np.zeros(19)
    lib().or_collide_cell(_d(_arr(f, 19)), rho0, omega_e, omega_o, _d(_arr(g, 3)), _d(out))
    return out


def fiber_axis(q):
    t = np.zeros(3)
    lib().or_fiber_axis(_d(_arr(q, 4)), _d(t))
    return t


SHAPES = {"cylinder": 0, "spherocylinder": 1}


def map_fibers(shape, X, q, length, radius, z_periodic=False, shapes=None):
    """shape = (nx, ny, nz); returns (pid[nz][ny][nx], overlaps).  shapes:
    per-fiber "cylinder"/"spherocylinder" (default all cylinders)."""
    nx, ny, nz = shape
    X = _arr(X).reshape(-1, 3)
    n = X.shape[0]
    pid = np.zeros((nz, ny, nx), np.int32)
    ov = np.zeros(1, np.int64)
    codes = np.array([SHAPES[k] if isinstance(k, str) else int(k) for k in
                      (shapes if shapes is not None else ["cylinder"] * n)], np.int32)
    lib().or_map_shapes(nx, ny, nz, int(z_periodic), n, _d(X), _d(_arr(q, 4 * n)),
                        _d(_arr(length, n)), _d(_arr(radius, n)), codes.ctypes.data_as(_ip),
                        pid.ctypes.data_as(_ip), ov.ctypes.data_as(_i64p))
    return pid, int(ov[0])


def body_inertia(shape, length, radius, rho):
    """(mass, I about the axis, I about a transverse axis through the centre)."""
    out = np.zeros(3)
    code = SHAPES[shape] if isinstance(shape, str) else int(shape)
    lib().or_body_inertia(code, float(length), float(radius), float(rho), _d(out))
    return out


def cell_inside(c, X, t, length, radius, shape="cylinder", dims=(1 << 20, 1 << 20, 1 << 20),
                z_periodic=True):
    """The cell-centre predicate for one cell and one fiber axis t."""
    code = SHAPES[shape] if isinstance(shape, str) else int(shape)
    return bool(lib().or_cell_inside_shape(_d(_arr(c, 3)), _d(_arr(X, 3)), _d(_arr(t, 3)),
                                           float(length), float(radius), code, dims[0], dims[1],
                                           dims[2], int(z_periodic)))


def set_threads(n):
    """OpenMP threads used by the following oracle steps."""
    lib().or_set_threads(int(n))


def get_threads():
    return int(lib().or_get_threads())


def set_mutation(code):
    """Plant a known mistake in the oracle (tests of the pins only); 0 clears it."""
    lib().or_set_mutation(int(code))


def rigid_step_implicit(state, mass, i_par, i_perp, F0, M0, A, B, Cm,
                        shape=(1 << 20, 1 << 20, 1 << 20), z_periodic=True):
    """Implicit step: solves (m + A) V' + B W' = m V + F0, B^T V' + (I + C) W' = Lang + M0.
    Returns (new state, applied F, applied M)."""
    out, Fa, Ma = np.zeros(16), np.zeros(3), np.zeros(3)
    nx, ny, nz = shape
    lib().or_rigid_step_implicit(_d(_arr(state, 16)), mass, i_par, i_perp, _d(_arr(F0, 3)),
                                 _d(_arr(M0, 3)), _d(_arr(A, 9)), _d(_arr(B, 9)), _d(_arr(Cm, 9)),
                                 nx, ny, nz, int(z_periodic), _d(out), _d(Fa), _d(Ma))
    return out, Fa, Ma


def rigid_step(state, mass, i_par, i_perp, F, M, shape=(1 << 20, 1 << 20, 1 << 20),
               z_periodic=True):
    """state = X3 q4 V3 W3 Lang3 (16 doubles) -> new state."""
    out = np.zeros(16)
    nx, ny, nz = shape
    lib().or_rigid_step(_d(_arr(state, 16)), mass, i_par, i_perp, _d(_arr(F, 3)),
                        _d(_arr(M, 3)), nx, ny, nz, int(z_periodic), _d(out))
    return out


# ---------------------------------------------------------------- coupled simulation
# coupling of the momentum-exchange force to the rigid-body update (or_params.coupling)
COUPLING = {"implicit": 0, "explicit": 1, "implicit_plain": 2}


def segment_closest(Xp, tp, hp, Xq, tq, hq):
    """Distance of two axis segments X + s t, |s| <= h, and the parameters s, u."""
    s, u = C.c_double(), C.c_double()
    d = lib().or_segment_closest(_d(_arr(Xp, 3)), _d(_arr(tp, 3)), float(hp), _d(_arr(Xq, 3)),
                                 _d(_arr(tq, 3)), float(hq), C.byref(s), C.byref(u))
    return d, s.value, u.value


def contact_pair(tp, hp, rp, dpq, tq, hq, rq, k, rng):
    """Contact force and torque on p and q (X_p at the origin, X_q at dpq); returns
    (gap, Fp, Mp, Fq, Mq)."""
    out = [np.zeros(3) for _ in range(4)]
    gap = lib().or_contact_pair(_d(_arr(tp, 3)), float(hp), float(rp), _d(_arr(dpq, 3)),
                                _d(_arr(tq, 3)), float(hq), float(rq), float(k), float(rng),
                                *[_d(o) for o in out])
    return (gap, *out)


WALL_KINDS = {"periodic": 0, "no-slip": 1, "free-slip": 2}


def wall_kind(v):
    """x/y wall argument: False (periodic), True or "no-slip", "free-slip"."""
    if isinstance(v, str):
        return WALL_KINDS[v]
    return 1 if v else 0


class Sim:
    """One coupled simulation held by the oracle."""

    def __init__(self, nx, ny, nz, tau=0.8, magic=3.0 / 16.0, wall_u=0.0, rho0=1.0,
                 z_periodic=False, srt=False, g=(0.0, 0.0, 0.0), init_couette=False,
                 coupling="implicit", stabilize=False, contact_k=0.0, contact_range=1.0,
                 x_walls=False, y_walls=False, z_free_slip=False):
        p = Params(nx, ny, nz, int(z_periodic), int(srt), tau, magic, rho0, wall_u,
                   (C.c_double * 3)(*g), int(init_couette), COUPLING[coupling], int(stabilize),
                   float(contact_k), float(contact_range), wall_kind(x_walls), wall_kind(y_walls),
                   int(bool(z_free_slip)))
        self.shape = (nx, ny, nz)
        self.ncell = nx * ny * nz
        self._h = lib().or_create(C.byref(p))
        if not self._h:
            raise MemoryError("oracle allocation failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def add_fiber(self, X, q, length, radius, density_ratio=1.0, V=(0, 0, 0), W=(0, 0, 0),
                  shape="cylinder", force=(0, 0, 0), torque=(0, 0, 0)):
        code = SHAPES[shape] if isinstance(shape, str) else int(shape)
        r = lib().or_add_fiber_ex(self._h, _d(_arr(X, 3)), _d(_arr(q, 4)), float(length),
                                  float(radius), float(density_ratio), _d(_arr(V, 3)),
                                  _d(_arr(W, 3)), code, _d(_arr(force, 3)), _d(_arr(torque, 3)))
        if r < 0:
            raise ValueError("oracle rejected the fiber (code %d)" % r)
        return r

    def set_kinematics(self, fid, traj):
        t = _arr(traj).reshape(-1, 13)
        lib().or_set_kinematics(self._h, fid, _d(t), t.shape[0])

    def set_correction(self, fid, dF, dM):
        """Add dF, dM to fiber fid's force and torque in the next step only."""
        lib().or_set_correction(self._h, fid, _d(_arr(dF, 3)), _d(_arr(dM, 3)))

    def step(self, n=1):
        lib().or_step(self._h, int(n))

    @property
    def nfibers(self):
        return lib().or_nfibers(self._h)

    @property
    def steps_done(self):
        return lib().or_steps_done(self._h)

    @property
    def overlaps(self):
        return lib().or_overlaps(self._h)

    def mean_velocity(self):
        """Mean fluid velocity of the current state and the fluid cell count."""
        u = np.zeros(3)
        n = lib().or_mean_velocity(self._h, _d(u))
        return u, int(n)

    def populations(self):
        nx, ny, nz = self.shape
        f = np.zeros((19, nz, ny, nx))
        lib().or_get_populations(self._h, _d(f))
        return f

    def set_populations(self, f):
        f = _arr(f, 19 * self.ncell)
        lib().or_set_populations(self._h, _d(f))

    def fields(self):
        nx, ny, nz = self.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        flags = np.zeros((nz, ny, nx), np.uint8)
        pid = np.zeros((nz, ny, nx), np.int32)
        lib().or_get_fields(self._h, _d(rho), _d(u), flags.ctypes.data_as(_u8p),
                            pid.ctypes.data_as(_ip))
        return rho, u, flags, pid

    def fiber_state(self):
        n = self.nfibers
        X, q, V, W = np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3)), np.zeros((n, 3))
        lib().or_get_fiber_state(self._h, _d(X), _d(q), _d(V), _d(W))
        return X, q, V, W

    def force_torque(self):
        n = self.nfibers
        F, M = np.zeros((n, 3)), np.zeros((n, 3))
        lib().or_get_force_torque(self._h, _d(F), _d(M))
        return F, M

    def exchange_sums(self):
        """Last step's sums per fiber: dict of F, M (direct), F0, M0 [n][3] and A, B, C [n][3][3]."""
        n = self.nfibers
        out = np.zeros((n, 39))
        lib().or_get_exchange_sums(self._h, _d(out))
        return {"F": out[:, 0:3], "M": out[:, 3:6], "F0": out[:, 6:9], "M0": out[:, 9:12],
                "A": out[:, 12:21].reshape(n, 3, 3), "B": out[:, 21:30].reshape(n, 3, 3),
                "C": out[:, 30:39].reshape(n, 3, 3)}

    def history(self, first=0, count=None):
        """[steps][nfibers][19]: F3 M3 X3 q4 V3 W3 after each step."""
        n = self.nfibers
        if count is None:
            count = self.steps_done - first
        out = np.zeros((max(count, 0), n, 19))
        got = lib().or_get_history(self._h, first, count, _d(out))
        return out[:got]
