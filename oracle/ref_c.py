"""ctypes front end of the plain C FP64 oracle (``ref_lbm.c``).

Test infrastructure only (see ``oracle/__init__.py``).  ``build()`` compiles
the C file with gcc/OpenMP into ``oracle/liboracle_lbm.so``; the functions
below marshal numpy arrays and call it.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import d3q19 as L

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ref_lbm.c")
LIB = os.path.join(HERE, "liboracle_lbm.so")


def build(force=False):
    """Compile the oracle (plain gcc, IEEE arithmetic: no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-D_DEFAULT_SOURCE", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("smag_form", ctypes.c_int32),
        ("tau0", ctypes.c_double), ("C", ctypes.c_double), ("rho0", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_pi", ctypes.c_double), ("s_m", ctypes.c_double),
        ("n_modes", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
        ("mode_k", ctypes.POINTER(ctypes.c_int32)),
        ("mode_amp", ctypes.POINTER(ctypes.c_double)),
        ("mode_phase", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        _lib.orc_step.argtypes = [pp, dp, dp, ctypes.c_int64]
        _lib.orc_step.restype = ctypes.c_int
        _lib.orc_fields.argtypes = [pp, dp, dp, dp, dp]
        _lib.orc_fields.restype = None
        _lib.orc_init.argtypes = [pp, ctypes.c_int, ctypes.c_double, ctypes.c_uint64, dp]
        _lib.orc_init.restype = ctypes.c_int
        _lib.orc_collide_cell.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        _lib.orc_collide_cell.restype = None
        _lib.orc_force_at.argtypes = [pp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        _lib.orc_force_at.restype = None
        _lib.orc_splitmix64.argtypes = [ctypes.c_uint64]
        _lib.orc_splitmix64.restype = ctypes.c_uint64
        _lib.orc_minv.argtypes = [dp]
        _lib.orc_minv.restype = None
        _lib.orc_num_threads.argtypes = []
        _lib.orc_num_threads.restype = ctypes.c_int
    return _lib


def _dptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Lattice:
    """Parameters of one oracle lattice; keeps the mode arrays alive."""

    def __init__(self, shape, tau0, C, modes=(), smag_form=0, rho0=1.0,
                 s_e=L.S_E, s_eps=L.S_EPS, s_q=L.S_Q, s_pi=L.S_PI, s_m=L.S_M, tau_mode=0):
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        modes = list(modes)
        n = len(modes)
        self._k = np.ascontiguousarray(
            np.array([m[0] for m in modes], dtype=np.int32).reshape(n, 3))
        self._amp = np.ascontiguousarray(
            np.array([m[1] for m in modes], dtype=np.float64).reshape(n, 3))
        self._ph = np.ascontiguousarray(np.array([m[2] for m in modes], dtype=np.float64))
        self.p = _Params(nx, ny, nz, smag_form, tau0, C, rho0, s_e, s_eps, s_q, s_pi, s_m,
                         n, tau_mode,
                         self._k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         self._amp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self._ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    @property
    def ncell(self):
        nz, ny, nx = self.shape
        return nx * ny * nz

    def init(self, kind, amp, seed=0):
        f = np.empty((19,) + self.shape)
        rc = lib().orc_init(ctypes.byref(self.p), kind, amp, seed, _dptr(f))
        if rc != 0:
            raise ValueError("orc_init failed")
        return f

    def step(self, f, nsteps=1):
        """Return f advanced by nsteps (the input array is not modified)."""
        f = np.ascontiguousarray(f, dtype=np.float64).copy()
        work = np.empty_like(f)
        rc = lib().orc_step(ctypes.byref(self.p), _dptr(f), _dptr(work), nsteps)
        if rc != 0:
            raise ValueError("orc_step failed")
        return f

    def fields(self, f):
        """rho (nz,ny,nx), u (3,nz,ny,nx), tau_e (nz,ny,nx) of state f."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = np.empty(self.shape)
        u = np.empty((3,) + self.shape)
        tau = np.empty(self.shape)
        lib().orc_fields(ctypes.byref(self.p), _dptr(f), _dptr(rho), _dptr(u), _dptr(tau))
        return rho, u, tau

    def force_at(self, x, y, z):
        F = np.zeros(3)
        lib().orc_force_at(ctypes.byref(self.p), x, y, z, _dptr(F))
        return F

    def collide_cell(self, fcell, F):
        fcell = np.ascontiguousarray(fcell, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.float64)
        out = np.empty(19)
        rho = np.zeros(1)
        u = np.zeros(3)
        tau = np.zeros(1)
        lib().orc_collide_cell(ctypes.byref(self.p), _dptr(fcell), _dptr(F), _dptr(out),
                               _dptr(rho), _dptr(u), _dptr(tau))
        return out, rho[0], u, tau[0]


def splitmix64(v):
    return int(lib().orc_splitmix64(v))


def minv():
    out = np.empty((19, 19))
    lib().orc_minv(_dptr(out))
    return out


def num_threads():
    return int(lib().orc_num_threads())
