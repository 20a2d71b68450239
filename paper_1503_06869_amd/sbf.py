"""ctypes binding of the slender-body formulation (include/sbf.h): argument
marshalling only; every step runs in the library's kernels (liblbmfib.so).
Raises when the library has not been built."""
import ctypes as C

import numpy as np

from . import lbm

EXPORTED_SBF = [
    "sbf_params_default", "sbf_create", "sbf_destroy", "sbf_last_error", "sbf_set_fibers",
    "sbf_solve", "sbf_get_velocities", "sbf_get_coefficients", "sbf_step", "sbf_get_state",
    "sbf_get_stats", "sbf_enable_timing", "sbf_get_timing",
]


class sbf_params(C.Structure):
    _fields_ = [("max_fibers", C.c_int32), ("nmodes", C.c_int32), ("nq", C.c_int32),
                ("gmres_restart", C.c_int32), ("gmres_maxit", C.c_int32), ("reserved", C.c_int32),
                ("length", C.c_double), ("eps", C.c_double), ("mu", C.c_double),
                ("gmres_tol", C.c_double), ("stream", C.c_void_p)]


_sig_done = False
_dp = C.POINTER(C.c_double)


def _lib():
    global _sig_done
    L = lbm.load()
    if not _sig_done:
        vp = C.c_void_p
        sig = {
            "sbf_params_default": ([C.POINTER(sbf_params)], C.c_int),
            "sbf_create": ([C.POINTER(sbf_params), C.POINTER(vp)], C.c_int),
            "sbf_destroy": ([vp], C.c_int),
            "sbf_last_error": ([vp], C.c_char_p),
            "sbf_set_fibers": ([vp, C.c_int32, _dp, _dp, _dp, _dp], C.c_int),
            "sbf_solve": ([vp], C.c_int),
            "sbf_get_velocities": ([vp, _dp, _dp], C.c_int),
            "sbf_get_coefficients": ([vp, _dp], C.c_int),
            "sbf_step": ([vp, C.c_int64, C.c_double], C.c_int),
            "sbf_get_state": ([vp, _dp, _dp], C.c_int),
            "sbf_get_stats": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int64)],
                              C.c_int),
            "sbf_enable_timing": ([vp, C.c_int32], C.c_int),
            "sbf_get_timing": ([vp, _dp, C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int64)], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _sig_done = True
    return L


def _f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))
    return a


class SBF:
    """M slender fibers of length L and slenderness eps in free space
    (Sec. 3 of the paper), on the GPU."""

    def __init__(self, max_fibers, length, eps, mu=1.0, nmodes=5, nq=16, gmres_tol=1e-12,
                 gmres_restart=30, gmres_maxit=200, stream=None):
        L = _lib()
        p = sbf_params()
        L.sbf_params_default(C.byref(p))
        p.max_fibers, p.nmodes, p.nq = int(max_fibers), int(nmodes), int(nq)
        p.gmres_restart, p.gmres_maxit = int(gmres_restart), int(gmres_maxit)
        p.length, p.eps, p.mu, p.gmres_tol = float(length), float(eps), float(mu), float(gmres_tol)
        p.stream = stream
        h = C.c_void_p()
        r = L.sbf_create(C.byref(p), C.byref(h))
        if r != lbm.LBM_OK:
            raise lbm.LBMError(r, "sbf_create failed")
        self._h = h
        self.N = int(nmodes)
        self.m = 0

    def _chk(self, r):
        if r not in (lbm.LBM_OK,):
            raise lbm.LBMError(r, _lib().sbf_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) and lbm._lib is not None:
            lbm._lib.sbf_destroy(self._h)
            self._h = None

    __del__ = close

    def set_fibers(self, X, p, F=None, M=None):
        X = _f64(X, (-1, 3))
        m = X.shape[0]
        p = _f64(p, (m, 3))
        Fa = _f64(F, (m, 3)) if F is not None else None
        Ma = _f64(M, (m, 3)) if M is not None else None
        self._chk(_lib().sbf_set_fibers(self._h, m, X.ctypes.data_as(_dp), p.ctypes.data_as(_dp),
                                        Fa.ctypes.data_as(_dp) if Fa is not None else None,
                                        Ma.ctypes.data_as(_dp) if Ma is not None else None))
        self.m = m

    def solve(self):
        self._chk(_lib().sbf_solve(self._h))

    def velocities(self):
        V, W = np.zeros((self.m, 3)), np.zeros((self.m, 3))
        self._chk(_lib().sbf_get_velocities(self._h, V.ctypes.data_as(_dp), W.ctypes.data_as(_dp)))
        return V, W

    def coefficients(self):
        a = np.zeros((self.m, self.N, 3))
        self._chk(_lib().sbf_get_coefficients(self._h, a.ctypes.data_as(_dp)))
        return a

    def step(self, n, dt):
        self._chk(_lib().sbf_step(self._h, int(n), float(dt)))

    def state(self):
        X, p = np.zeros((self.m, 3)), np.zeros((self.m, 3))
        self._chk(_lib().sbf_get_state(self._h, X.ctypes.data_as(_dp), p.ctypes.data_as(_dp)))
        return X, p

    def stats(self):
        it, res, st = C.c_int32(), C.c_double(), C.c_int64()
        self._chk(_lib().sbf_get_stats(self._h, C.byref(it), C.byref(res), C.byref(st)))
        return {"iterations": it.value, "residual": res.value, "steps": st.value}

    def enable_timing(self, on=True):
        self._chk(_lib().sbf_enable_timing(self._h, int(bool(on))))

    def timing(self):
        """(moment kernel ms, launches, moment-matrix GEMV ms, launches) since enabling."""
        tm, tg = C.c_double(), C.c_double()
        nm, ng = C.c_int64(), C.c_int64()
        self._chk(_lib().sbf_get_timing(self._h, C.byref(tm), C.byref(nm), C.byref(tg), C.byref(ng)))
        return tm.value, nm.value, tg.value, ng.value
