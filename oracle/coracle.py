"""ctypes wrapper of the plain-C FP64 oracle (oracle/coracle.c).

TEST INFRASTRUCTURE ONLY (tests/, __graft_entry__.smoke(), bench.py cpu_baseline).
Same interface as oracle.tfan_oracle.Oracle: init_fields, step, get_fields."""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("n_sub", ctypes.c_int)] + [
        (k, ctypes.c_double) for k in ("rho0", "tau_a", "tau_p", "gamma", "A_ch", "kappa", "M",
                                       "A0", "gamma_ldg", "K", "lam", "Gamma", "zeta")]


def _load():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "libcoracle.so")
        if not os.path.exists(path):
            from oracle.build_coracle import build
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oc_create.restype = ctypes.c_void_p
        lib.oc_create.argtypes = [ctypes.POINTER(_Params)]
        lib.oc_destroy.argtypes = [ctypes.c_void_p]
        lib.oc_init.argtypes = [ctypes.c_void_p] + [dp] * 5
        lib.oc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.oc_fields.argtypes = [ctypes.c_void_p] + [dp] * 7
        lib.oc_threads.restype = ctypes.c_int
        lib.oc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().oc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of later steps (timing only: results do not depend on it)."""
    _load().oc_set_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class COracle:
    def __init__(self, params: dict):
        lib = _load()
        p = _Params()
        for name, typ in _Params._fields_:
            setattr(p, name, int(params[name]) if typ is ctypes.c_int else float(params[name]))
        if p.tau_a <= 0.5 or p.tau_p <= 0.5 or p.n_sub < 1:
            raise ValueError("tau must exceed 1/2 and n_sub must be >= 1")
        self.nx, self.ny = p.nx, p.ny
        self._h = lib.oc_create(ctypes.byref(p))
        self.step_count = 0

    def init_fields(self, phi, qxx, qxy, u_a=None, u_p=None):
        s = (self.ny, self.nx)
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(s) for a in (phi, qxx, qxy)]
        us = [None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape((2,) + s)
              for u in (u_a, u_p)]
        _load().oc_init(self._h, *[_ptr(a) for a in arrs + us])
        self.step_count = 0

    def step(self, n: int = 1):
        _load().oc_step(self._h, int(n))
        self.step_count += int(n)

    def get_fields(self) -> dict:
        s = (self.ny, self.nx)
        out = dict(phi=np.empty(s), qxx=np.empty(s), qxy=np.empty(s), u_a=np.empty((2,) + s),
                   u_p=np.empty((2,) + s), rho_a=np.empty(s), rho_p=np.empty(s))
        _load().oc_fields(self._h, *[_ptr(out[k]) for k in ("phi", "qxx", "qxy", "u_a", "u_p", "rho_a", "rho_p")])
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            _load().oc_destroy(self._h)
            self._h = None
