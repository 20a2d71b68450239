"""Thin ctypes binding of the C ABI in include/lbm.h and include/lbm_batch.h
(argument marshalling only).

The functions keep the C names (``lbm_create``, ``lbm_step``,
``lbm_batch_step``, ...).  The ``Context`` class wraps one lattice, the
``Batch`` class many independent one-fiber cases, with numpy in/out arrays.
Every step of the method runs in the HIP kernels of ``liblbmfib.so``; if
that library is missing, ``load()`` raises (there is no fallback).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmfib.so")

LBM_OK, LBM_E_ARG, LBM_E_NOMEM, LBM_E_HIP, LBM_E_GEOM, LBM_E_UNSTABLE, LBM_E_STATE = range(7)
LBM_TRT, LBM_SRT = 0, 1
LBM_F32, LBM_F16DEV, LBM_BF16DEV, LBM_F64 = 0, 1, 2, 3
LBM_INIT_REST, LBM_INIT_COUETTE = 0, 1
LBM_COUPLING_IMPLICIT, LBM_COUPLING_EXPLICIT, LBM_COUPLING_IMPLICIT_PLAIN = 0, 1, 2
COUPLING = {"implicit": LBM_COUPLING_IMPLICIT, "explicit": LBM_COUPLING_EXPLICIT,
            "implicit_plain": LBM_COUPLING_IMPLICIT_PLAIN}

STORAGE = {"f32": LBM_F32, "f16": LBM_F16DEV, "bf16": LBM_BF16DEV, "f64": LBM_F64}

EXPORTED = [
    "lbm_params_default", "lbm_create", "lbm_destroy", "lbm_last_error", "lbm_lattice",
    "lbm_add_fiber", "lbm_set_fiber_kinematics", "lbm_step", "lbm_sync",
    "lbm_get_force_torque", "lbm_get_fields", "lbm_get_fiber_state", "lbm_set_fiber_state",
    "lbm_get_history", "lbm_get_populations", "lbm_set_populations", "lbm_get_info",
    "lbm_enable_sweep_timing", "lbm_get_sweep_time", "lbm_copy_bytes", "lbm_get_mean_velocity",
    "lbm_get_params", "lbm_save", "lbm_load", "lbm_get_fields_static",
]
EXPORTED_BATCH = [
    "lbm_batch_params_default", "lbm_batch_create", "lbm_batch_destroy", "lbm_batch_last_error",
    "lbm_batch_set_kinematics", "lbm_batch_autotune", "lbm_batch_set_config", "lbm_batch_step",
    "lbm_batch_sync", "lbm_batch_get_force_torque", "lbm_batch_get_fiber_state",
    "lbm_batch_get_history", "lbm_batch_get_fields", "lbm_batch_get_populations",
    "lbm_batch_get_info",
]
EXPORTED_MLP = [
    "lbm_mlp_create", "lbm_mlp_destroy", "lbm_mlp_last_error", "lbm_mlp_set_params",
    "lbm_mlp_get_params", "lbm_mlp_set_norm", "lbm_mlp_forward", "lbm_mlp_loss_grad",
    "lbm_mlp_adam", "lbm_mlp_train", "lbm_set_closure", "lbm_get_closure_stats",
    "lbm_sample_features", "lbm_batch_sample_features",
]
MLP_IN, MLP_OUT, MLP_NPARAM = 247, 6, 20422


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("z_periodic", C.c_int32), ("collision", C.c_int32),
                ("tau", C.c_double), ("magic", C.c_double), ("wall_u", C.c_double),
                ("rho0", C.c_double), ("body_force", C.c_double * 3),
                ("storage", C.c_int32), ("init_profile", C.c_int32), ("coupling", C.c_int32),
                ("fp16_scale_log2", C.c_int32), ("history_capacity", C.c_int64),
                ("stream", C.c_void_p), ("sweep_grid", C.c_int32), ("q_pad", C.c_int32),
                ("stabilize", C.c_int32), ("z_free_slip", C.c_int32),
                ("contact_stiffness", C.c_double), ("contact_range", C.c_double),
                ("x_walls", C.c_int32), ("y_walls", C.c_int32)]


class lbm_fiber(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("quat", C.c_double * 4), ("length", C.c_double),
                ("radius", C.c_double), ("density_ratio", C.c_double),
                ("vel", C.c_double * 3), ("omega", C.c_double * 3),
                ("shape", C.c_int32), ("reserved", C.c_int32),
                ("force", C.c_double * 3), ("torque", C.c_double * 3)]


SHAPES = {"cylinder": 0, "spherocylinder": 1}


class lbm_info(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("nfibers", C.c_int32), ("parity", C.c_int32),
                ("boundary_cells", C.c_int64), ("overlap_events", C.c_int64),
                ("device_bytes", C.c_int64), ("population_bytes", C.c_int64)]


class lbm_batch_case(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("tau", C.c_double),
                ("wall_u", C.c_double), ("fiber", lbm_fiber)]


class lbm_batch_params(C.Structure):
    _fields_ = [("collision", C.c_int32), ("magic", C.c_double), ("rho0", C.c_double),
                ("storage", C.c_int32), ("init_profile", C.c_int32), ("coupling", C.c_int32),
                ("fp16_scale_log2", C.c_int32), ("history_capacity", C.c_int64),
                ("stream", C.c_void_p), ("threads", C.c_int32), ("bins", C.c_int32)]


class lbm_batch_tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("bins", C.c_int32), ("ms_per_step", C.c_double),
                ("from_cache", C.c_int32), ("trials", C.c_int32)]


class lbm_batch_info(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("ncases", C.c_int32), ("bins", C.c_int32),
                ("threads", C.c_int32), ("cells", C.c_int64), ("boundary_cells", C.c_int64),
                ("device_bytes", C.c_int64), ("population_bytes", C.c_int64)]


_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_lib = None


def load():
    """Load liblbmfib.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbmfib.so not built: run paper_1503_06869_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "lbm_params_default": ([C.POINTER(lbm_params)], C.c_int),
        "lbm_create": ([C.POINTER(lbm_params), C.POINTER(vp)], C.c_int),
        "lbm_destroy": ([vp], C.c_int),
        "lbm_last_error": ([vp], C.c_char_p),
        "lbm_lattice": ([C.POINTER(C.c_int32), _dp], C.c_int),
        "lbm_add_fiber": ([vp, C.POINTER(lbm_fiber), C.POINTER(C.c_int32)], C.c_int),
        "lbm_set_fiber_kinematics": ([vp, C.c_int32, _dp, C.c_int64], C.c_int),
        "lbm_step": ([vp, C.c_int64], C.c_int),
        "lbm_sync": ([vp], C.c_int),
        "lbm_get_force_torque": ([vp, _dp, _dp], C.c_int),
        "lbm_get_fields": ([vp, vp, vp, vp, vp, C.c_int32], C.c_int),
        "lbm_get_fields_static": ([vp, vp, vp, vp, vp], C.c_int),
        "lbm_get_fiber_state": ([vp, _dp, _dp, _dp, _dp], C.c_int),
        "lbm_set_fiber_state": ([vp, C.c_int32, _dp, _dp, _dp, _dp], C.c_int),
        "lbm_get_history": ([vp, C.c_int64, C.c_int64, _dp], C.c_int),
        "lbm_get_populations": ([vp, _dp], C.c_int),
        "lbm_set_populations": ([vp, _dp], C.c_int),
        "lbm_get_info": ([vp, C.POINTER(lbm_info)], C.c_int),
        "lbm_get_mean_velocity": ([vp, _dp, C.POINTER(C.c_int64)], C.c_int),
        "lbm_get_params": ([vp, C.POINTER(lbm_params)], C.c_int),
        "lbm_save": ([vp, C.c_char_p], C.c_int),
        "lbm_load": ([C.c_char_p, vp, C.POINTER(vp)], C.c_int),
        "lbm_enable_sweep_timing": ([vp, C.c_int32], C.c_int),
        "lbm_get_sweep_time": ([vp, _dp, C.POINTER(C.c_int64)], C.c_int),
        "lbm_copy_bytes": ([vp, vp, C.c_size_t, vp], C.c_int),
        "lbm_batch_params_default": ([C.POINTER(lbm_batch_params)], C.c_int),
        "lbm_batch_create": ([C.POINTER(lbm_batch_params), C.POINTER(lbm_batch_case), C.c_int32,
                              C.POINTER(vp)], C.c_int),
        "lbm_batch_destroy": ([vp], C.c_int),
        "lbm_batch_last_error": ([vp], C.c_char_p),
        "lbm_batch_set_kinematics": ([vp, C.c_int32, _dp, C.c_int64], C.c_int),
        "lbm_batch_autotune": ([vp, C.c_int32, C.c_char_p, C.POINTER(lbm_batch_tuning)], C.c_int),
        "lbm_batch_set_config": ([vp, C.c_int32, C.c_int32], C.c_int),
        "lbm_batch_step": ([vp, C.c_int64], C.c_int),
        "lbm_batch_sync": ([vp], C.c_int),
        "lbm_batch_get_force_torque": ([vp, _dp, _dp], C.c_int),
        "lbm_batch_get_fiber_state": ([vp, _dp, _dp, _dp, _dp], C.c_int),
        "lbm_batch_get_history": ([vp, C.c_int32, C.c_int64, C.c_int64, _dp], C.c_int),
        "lbm_batch_get_fields": ([vp, C.c_int32, vp, vp, vp, vp, C.c_int32], C.c_int),
        "lbm_batch_get_populations": ([vp, C.c_int32, _dp], C.c_int),
        "lbm_batch_get_info": ([vp, C.POINTER(lbm_batch_info)], C.c_int),
        "lbm_mlp_create": ([C.c_uint64, vp, C.POINTER(vp)], C.c_int),
        "lbm_mlp_destroy": ([vp], C.c_int),
        "lbm_mlp_last_error": ([vp], C.c_char_p),
        "lbm_mlp_set_params": ([vp, _fp], C.c_int),
        "lbm_mlp_get_params": ([vp, _fp, C.POINTER(C.c_uint16)], C.c_int),
        "lbm_mlp_set_norm": ([vp, _fp, _fp, _fp, _fp, _fp], C.c_int),
        "lbm_mlp_forward": ([vp, vp, C.c_int32, vp], C.c_int),
        "lbm_mlp_loss_grad": ([vp, vp, vp, C.c_int32, _dp, _fp], C.c_int),
        "lbm_mlp_adam": ([vp, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
        "lbm_mlp_train": ([vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_uint64, _dp],
                          C.c_int),
        "lbm_set_closure": ([vp, vp], C.c_int),
        "lbm_get_closure_stats": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
        "lbm_sample_features": ([vp, vp, C.c_int32], C.c_int),
        "lbm_batch_sample_features": ([vp, vp, C.c_int32], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm error %d: %s" % (code, msg))
        self.code = code


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def lattice():
    """(c[19][3], w[19]) in the library's population order."""
    c = np.zeros(57, np.int32)
    w = np.zeros(19)
    load().lbm_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)), _d(w))
    return c.reshape(19, 3), w


def copy_bytes(dst_ptr, src_ptr, nbytes, stream=None):
    r = load().lbm_copy_bytes(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), nbytes, C.c_void_p(stream or 0))
    if r != LBM_OK:
        raise LBMError(r, "copy failed")


WALLS = {"periodic": 0, "no-slip": 1, "free-slip": 2}


def _wall_code(v):
    if isinstance(v, str):
        return WALLS[v]
    return 1 if v else 0


class Context:
    """One lattice with its fibers (owns an lbm_ctx)."""

    def __init__(self, nx, ny, nz, tau=0.8, magic=3.0 / 16.0, wall_u=0.0, rho0=1.0,
                 z_periodic=False, collision="trt", storage="f32", init_couette=False,
                 coupling="implicit", body_force=(0.0, 0.0, 0.0), fp16_scale_log2=14,
                 history_capacity=4096, stream=None, sweep_grid=0, q_pad=-1, stabilize=False,
                 contact_k=0.0, contact_range=1.0, x_walls=False, y_walls=False, z_free_slip=False):
        """stabilize: momentum stabilization (subtract the mean fluid velocity
        in every equilibrium), for fully periodic boxes with forced particles.
        contact_k, contact_range: short-range repulsion between fibers (off at 0).
        x_walls, y_walls: walls on the x (y) faces instead of periodicity --
        True or "no-slip" (resting), "free-slip" (specular reflection).
        z_free_slip: the z walls (z_periodic False, wall_u 0) are free-slip."""
        L = load()
        p = lbm_params()
        L.lbm_params_default(C.byref(p))
        p.nx, p.ny, p.nz = nx, ny, nz
        p.z_periodic = int(bool(z_periodic))
        p.collision = LBM_SRT if collision == "srt" else LBM_TRT
        p.tau, p.magic, p.wall_u, p.rho0 = tau, magic, wall_u, rho0
        p.body_force = (C.c_double * 3)(*body_force)
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.init_profile = LBM_INIT_COUETTE if init_couette else LBM_INIT_REST
        p.coupling = COUPLING[coupling]
        p.fp16_scale_log2 = fp16_scale_log2
        p.history_capacity = history_capacity
        p.stream = stream
        p.sweep_grid = sweep_grid
        p.q_pad = q_pad
        p.stabilize = int(bool(stabilize))
        p.contact_stiffness = float(contact_k)
        p.contact_range = float(contact_range)
        p.x_walls = _wall_code(x_walls)
        p.y_walls = _wall_code(y_walls)
        p.z_free_slip = int(bool(z_free_slip))
        h = C.c_void_p()
        r = L.lbm_create(C.byref(p), C.byref(h))
        if r != LBM_OK:
            raise LBMError(r, "lbm_create failed")
        self._h = h
        self.shape = (nx, ny, nz)
        self.ncell = nx * ny * nz
        self.storage = p.storage
        self.nfibers = 0

    def _chk(self, r):
        if r != LBM_OK:
            raise LBMError(r, load().lbm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lbm_destroy(self._h)
            self._h = None

    __del__ = close

    def add_fiber(self, X, q, length, radius, density_ratio=1.0, V=(0, 0, 0), W=(0, 0, 0),
                  shape="cylinder", force=(0, 0, 0), torque=(0, 0, 0)):
        """shape: "cylinder" or "spherocylinder" (length including the caps);
        force, torque: constant external load added in every step."""
        f = _fiber_struct(X, q, length, radius, density_ratio, V, W, shape, force, torque)
        i = C.c_int32()
        self._chk(load().lbm_add_fiber(self._h, C.byref(f), C.byref(i)))
        self.nfibers += 1
        return i.value

    def set_kinematics(self, fid, traj):
        t = _f64(traj).reshape(-1, 13)
        self._chk(load().lbm_set_fiber_kinematics(self._h, fid, _d(t), t.shape[0]))

    def step(self, n=1):
        self._chk(load().lbm_step(self._h, int(n)))

    def sync(self):
        self._chk(load().lbm_sync(self._h))

    def force_torque(self):
        F, M = np.zeros((self.nfibers, 3)), np.zeros((self.nfibers, 3))
        self._chk(load().lbm_get_force_torque(self._h, _d(F), _d(M)))
        return F, M

    def fields(self):
        nx, ny, nz = self.shape
        dt = np.float64 if self.storage == LBM_F64 else np.float32
        rho = np.zeros((nz, ny, nx), dt)
        u = np.zeros((3, nz, ny, nx), dt)
        flags = np.zeros((nz, ny, nx), np.uint8)
        pid = np.zeros((nz, ny, nx), np.int32)
        self._chk(load().lbm_get_fields(self._h, rho.ctypes.data, u.ctypes.data, flags.ctypes.data,
                                        pid.ctypes.data, 0))
        return rho, u, flags, pid

    def fields_static(self):
        """As fields(), through lbm_get_fields_static (no device allocation)."""
        nx, ny, nz = self.shape
        dt = np.float64 if self.storage == LBM_F64 else np.float32
        rho = np.zeros((nz, ny, nx), dt)
        u = np.zeros((3, nz, ny, nx), dt)
        flags = np.zeros((nz, ny, nx), np.uint8)
        pid = np.zeros((nz, ny, nx), np.int32)
        self._chk(load().lbm_get_fields_static(self._h, rho.ctypes.data, u.ctypes.data,
                                               flags.ctypes.data, pid.ctypes.data))
        return rho, u, flags, pid

    def fields_to_device(self, rho_ptr, u_ptr):
        """Write rho and u into device buffers (e.g. torch tensors' data_ptr())."""
        self._chk(load().lbm_get_fields(self._h, C.c_void_p(rho_ptr), C.c_void_p(u_ptr), None,
                                        None, 1))

    def fiber_state(self):
        n = self.nfibers
        X, q, V, W = np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3)), np.zeros((n, 3))
        self._chk(load().lbm_get_fiber_state(self._h, _d(X), _d(q), _d(V), _d(W)))
        return X, q, V, W

    def set_fiber_state(self, fid, X, q, V=(0, 0, 0), W=(0, 0, 0)):
        self._chk(load().lbm_set_fiber_state(self._h, fid, _d(_f64(X, 3)), _d(_f64(q, 4)),
                                             _d(_f64(V, 3)), _d(_f64(W, 3))))

    def history(self, first, count):
        out = np.zeros((count, self.nfibers, 19))
        self._chk(load().lbm_get_history(self._h, first, count, _d(out)))
        return out

    def populations(self):
        nx, ny, nz = self.shape
        f = np.zeros((19, nz, ny, nx))
        self._chk(load().lbm_get_populations(self._h, _d(f)))
        return f

    def set_populations(self, f):
        self._chk(load().lbm_set_populations(self._h, _d(_f64(f, 19 * self.ncell))))

    def save(self, path):
        """Write a checkpoint of the whole state to path."""
        self._chk(load().lbm_save(self._h, str(path).encode()))

    @classmethod
    def load_checkpoint(cls, path, stream=None):
        """A context restored from a checkpoint written by save()."""
        L = load()
        h = C.c_void_p()
        r = L.lbm_load(str(path).encode(), stream, C.byref(h))
        if r != LBM_OK:
            raise LBMError(r, "lbm_load failed for %s" % path)
        self = cls.__new__(cls)
        self._h = h
        p = lbm_params()
        self._chk(L.lbm_get_params(h, C.byref(p)))
        self.shape = (p.nx, p.ny, p.nz)
        self.ncell = p.nx * p.ny * p.nz
        self.storage = p.storage
        i = lbm_info()
        self._chk(L.lbm_get_info(h, C.byref(i)))
        self.nfibers = i.nfibers
        return self

    def mean_velocity(self):
        """Mean fluid velocity the next step subtracts, and the fluid cell count
        (contexts created with stabilize=True)."""
        u, n = np.zeros(3), C.c_int64()
        self._chk(load().lbm_get_mean_velocity(self._h, _d(u), C.byref(n)))
        return u, n.value

    def info(self):
        i = lbm_info()
        self._chk(load().lbm_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in lbm_info._fields_}

    def set_closure(self, mlp):
        """Attach a trained Mlp (None detaches); the Mlp must outlive the use."""
        self._closure = mlp
        self._chk(load().lbm_set_closure(self._h, mlp._h if mlp is not None else None))

    def closure_stats(self):
        a, f = C.c_int64(), C.c_int64()
        self._chk(load().lbm_get_closure_stats(self._h, C.byref(a), C.byref(f)))
        return a.value, f.value

    def features(self):
        out = np.zeros((self.nfibers, MLP_IN), np.float32)
        self._chk(load().lbm_sample_features(self._h, out.ctypes.data, 0))
        return out

    def enable_sweep_timing(self, on=True):
        self._chk(load().lbm_enable_sweep_timing(self._h, int(bool(on))))

    def sweep_time(self):
        ms = C.c_double()
        n = C.c_int64()
        self._chk(load().lbm_get_sweep_time(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def _fiber_struct(X, q, length, radius, density_ratio=1.0, V=(0, 0, 0), W=(0, 0, 0), shape="cylinder",
                  force=(0, 0, 0), torque=(0, 0, 0)):
    f = lbm_fiber()
    f.center = (C.c_double * 3)(*_f64(X, 3))
    f.quat = (C.c_double * 4)(*_f64(q, 4))
    f.length, f.radius, f.density_ratio = float(length), float(radius), float(density_ratio)
    f.vel = (C.c_double * 3)(*_f64(V, 3))
    f.omega = (C.c_double * 3)(*_f64(W, 3))
    f.shape = SHAPES[shape] if isinstance(shape, str) else int(shape)
    f.reserved = 0
    f.force = (C.c_double * 3)(*_f64(force, 3))
    f.torque = (C.c_double * 3)(*_f64(torque, 3))
    return f


class Batch:
    """Many independent one-fiber shear cells advanced by one persistent
    launch (owns an lbm_batch).  ``cases``: objects with nx, ny, nz, tau,
    wall_u and fibers[0] (X, q, length, radius, density_ratio, V, W, and
    optionally shape, force, torque)."""

    def __init__(self, cases, storage="f32", collision="trt", magic=3.0 / 16.0, rho0=1.0,
                 init_couette=True, coupling="implicit", fp16_scale_log2=14,
                 history_capacity=4096, stream=None, threads=0, bins=0):
        L = load()
        p = lbm_batch_params()
        L.lbm_batch_params_default(C.byref(p))
        p.collision = LBM_SRT if collision == "srt" else LBM_TRT
        p.magic, p.rho0 = magic, rho0
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.init_profile = LBM_INIT_COUETTE if init_couette else LBM_INIT_REST
        p.coupling = COUPLING[coupling]
        p.fp16_scale_log2 = fp16_scale_log2
        p.history_capacity = history_capacity
        p.stream = stream
        p.threads, p.bins = threads, bins
        arr = (lbm_batch_case * len(cases))()
        for i, sc in enumerate(cases):
            fb = sc.fibers[0]
            arr[i].nx, arr[i].ny, arr[i].nz = sc.nx, sc.ny, sc.nz
            arr[i].tau, arr[i].wall_u = sc.tau, sc.wall_u
            arr[i].fiber = _fiber_struct(fb.X, fb.q, fb.length, fb.radius, fb.density_ratio, fb.V, fb.W,
                                         getattr(fb, "shape", "cylinder"), getattr(fb, "force", (0, 0, 0)),
                                         getattr(fb, "torque", (0, 0, 0)))
        h = C.c_void_p()
        r = L.lbm_batch_create(C.byref(p), arr, len(cases), C.byref(h))
        if r != LBM_OK:
            raise LBMError(r, L.lbm_batch_last_error(None).decode())
        self._h = h
        self.ncases = len(cases)
        self.shapes = [(sc.nx, sc.ny, sc.nz) for sc in cases]
        self.storage = p.storage

    def _chk(self, r):
        if r != LBM_OK:
            raise LBMError(r, load().lbm_batch_last_error(self._h).decode())

    def close(self):
        # _lib is None only during interpreter shutdown; then nothing is freed
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lbm_batch_destroy(self._h)
            self._h = None

    __del__ = close

    def set_kinematics(self, c, traj):
        t = _f64(traj).reshape(-1, 13)
        self._chk(load().lbm_batch_set_kinematics(self._h, c, _d(t), t.shape[0]))

    def autotune(self, trial_steps=10, cache_path=None):
        t = lbm_batch_tuning()
        cp = cache_path.encode() if cache_path else None
        self._chk(load().lbm_batch_autotune(self._h, trial_steps, cp, C.byref(t)))
        return {k: getattr(t, k) for k, _ in lbm_batch_tuning._fields_}

    def set_config(self, threads=0, bins=0):
        self._chk(load().lbm_batch_set_config(self._h, threads, bins))

    def step(self, n=1):
        self._chk(load().lbm_batch_step(self._h, int(n)))

    def sync(self):
        self._chk(load().lbm_batch_sync(self._h))

    def force_torque(self):
        F, M = np.zeros((self.ncases, 3)), np.zeros((self.ncases, 3))
        self._chk(load().lbm_batch_get_force_torque(self._h, _d(F), _d(M)))
        return F, M

    def fiber_state(self):
        n = self.ncases
        X, q, V, W = np.zeros((n, 3)), np.zeros((n, 4)), np.zeros((n, 3)), np.zeros((n, 3))
        self._chk(load().lbm_batch_get_fiber_state(self._h, _d(X), _d(q), _d(V), _d(W)))
        return X, q, V, W

    def history(self, c, first, count):
        out = np.zeros((count, 19))
        self._chk(load().lbm_batch_get_history(self._h, c, first, count, _d(out)))
        return out

    def fields(self, c):
        nx, ny, nz = self.shapes[c]
        dt = np.float64 if self.storage == LBM_F64 else np.float32
        rho = np.zeros((nz, ny, nx), dt)
        u = np.zeros((3, nz, ny, nx), dt)
        flags = np.zeros((nz, ny, nx), np.uint8)
        pid = np.zeros((nz, ny, nx), np.int32)
        self._chk(load().lbm_batch_get_fields(self._h, c, rho.ctypes.data, u.ctypes.data,
                                              flags.ctypes.data, pid.ctypes.data, 0))
        return rho, u, flags, pid

    def populations(self, c):
        nx, ny, nz = self.shapes[c]
        f = np.zeros((19, nz, ny, nx))
        self._chk(load().lbm_batch_get_populations(self._h, c, _d(f)))
        return f

    def features(self):
        out = np.zeros((self.ncases, MLP_IN), np.float32)
        self._chk(load().lbm_batch_sample_features(self._h, out.ctypes.data, 0))
        return out

    def features_to_device(self, ptr):
        self._chk(load().lbm_batch_sample_features(self._h, C.c_void_p(ptr), 1))

    def info(self):
        i = lbm_batch_info()
        self._chk(load().lbm_batch_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in lbm_batch_info._fields_}


def _f32(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


class Mlp:
    """The closure network (owns an lbm_mlp).  Device arrays are passed as
    data pointers (e.g. torch tensors' data_ptr())."""

    def __init__(self, seed=0, stream=None):
        h = C.c_void_p()
        r = load().lbm_mlp_create(seed, stream, C.byref(h))
        if r != LBM_OK:
            raise LBMError(r, "lbm_mlp_create failed")
        self._h = h

    def _chk(self, r):
        if r != LBM_OK:
            raise LBMError(r, load().lbm_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lbm_mlp_destroy(self._h)
            self._h = None

    __del__ = close

    def set_params(self, w):
        a = _f32(w, MLP_NPARAM)
        self._chk(load().lbm_mlp_set_params(self._h, a.ctypes.data_as(_fp)))

    def params(self):
        w = np.zeros(MLP_NPARAM, np.float32)
        wb = np.zeros(MLP_NPARAM, np.uint16)
        self._chk(load().lbm_mlp_get_params(self._h, w.ctypes.data_as(_fp),
                                            wb.ctypes.data_as(C.POINTER(C.c_uint16))))
        return w, wb

    def set_norm(self, in_mean=None, in_inv_std=None, out_scale=None, env_min=None, env_max=None):
        def p(a, n):
            return None if a is None else _f32(a, n).ctypes.data_as(_fp)
        keep = [None if a is None else _f32(a) for a in (in_mean, in_inv_std, out_scale, env_min, env_max)]
        self._chk(load().lbm_mlp_set_norm(self._h, p(keep[0], MLP_IN), p(keep[1], MLP_IN),
                                          p(keep[2], MLP_OUT), p(keep[3], MLP_IN), p(keep[4], MLP_IN)))

    def forward(self, x_ptr, n, y_ptr):
        self._chk(load().lbm_mlp_forward(self._h, C.c_void_p(x_ptr), n, C.c_void_p(y_ptr)))

    def loss_grad(self, x_ptr, t_ptr, n, want_grad=True):
        loss = C.c_double()
        g = np.zeros(MLP_NPARAM, np.float32) if want_grad else None
        self._chk(load().lbm_mlp_loss_grad(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), n, C.byref(loss),
                                           g.ctypes.data_as(_fp) if g is not None else None))
        return loss.value, g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(load().lbm_mlp_adam(self._h, lr, beta1, beta2, eps))

    def train(self, x_ptr, t_ptr, n, epochs, batch, lr, shuffle_seed=0):
        losses = np.zeros(epochs)
        self._chk(load().lbm_mlp_train(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), n, epochs, batch, lr,
                                       shuffle_seed, _d(losses)))
        return losses
