"""Thin ctypes binding of liblbm.so (see ``include/lbm.h``).

The functions ``lbm_*`` below carry the C names and only marshal arguments:
every step of the method runs in the HIP kernels behind the C-ABI.  torch is
used for two things only: the device buffer that holds the population state
(``torch.empty(..., dtype=torch.uint8, device="cuda")``) and the HIP stream
(``torch.cuda.current_stream().cuda_stream``).

Loading fails loudly (``RuntimeError``) when the library has not been built;
there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_ERR_INVALID_ARG, LBM_ERR_OUT_OF_MEMORY = 0, -1, -2
LBM_ERR_DEVICE, LBM_ERR_UNSTABLE, LBM_ERR_STATE = -3, -4, -5
LBM_FP64, LBM_FP32, LBM_FP16_DEV, LBM_BF16_DEV = 0, 1, 2, 3
LBM_STREAM_AA, LBM_STREAM_AB = 0, 1
LBM_INIT_NOISE, LBM_INIT_TGV3D, LBM_INIT_TGV2D, LBM_INIT_SHEAR, LBM_INIT_REST = 0, 1, 2, 3, 4

PRECISION = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16": LBM_FP16_DEV, "bf16": LBM_BF16_DEV}
STREAMING = {"aa": LBM_STREAM_AA, "ab": LBM_STREAM_AB}

# C-ABI entry points every build must export (checked by the CPU tests).
EXPORTS = (
    "lbm_config_default", "lbm_required_bytes", "lbm_create", "lbm_init_seeded",
    "lbm_init_velocity", "lbm_step",
    "lbm_stream_only",
    "lbm_moments", "lbm_kt_stats", "lbm_kt_field", "lbm_kt_slice", "lbm_get_populations",
    "lbm_set_populations", "lbm_sample_populations", "lbm_synchronize", "lbm_set_stream",
    "lbm_steps_done",
    "lbm_num_cells", "lbm_destroy", "lbm_status_string", "lbm_last_error",
    "lbm_batch_create", "lbm_batch_step", "lbm_batch_last_error", "lbm_batch_destroy",
    "lbm_theta_histogram_noalloc",
    "lbm_state_bytes", "lbm_save_state", "lbm_load_state",
    "lbm_theta_histogram", "lbm_spectrum", "lbm_spectra_1d", "lbm_structure_functions",
    "lbm_snapshot_begin", "lbm_snapshot_end",
    "lbm_turbulence",
)


class lbm_force_mode(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
                ("amp", ctypes.c_double * 3), ("phase", ctypes.c_double)]


class lbm_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("streaming", ctypes.c_int32),
        ("smag_form", ctypes.c_int32),
        ("tau0", ctypes.c_double), ("smag_C", ctypes.c_double), ("rho0", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_pi", ctypes.c_double), ("s_m", ctypes.c_double),
        ("storage_scale", ctypes.c_double),
        ("n_force_modes", ctypes.c_int32), ("steps_per_graph", ctypes.c_int32),
        ("temporal_block", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
        ("force_modes", ctypes.POINTER(lbm_force_mode)),
        ("hip_stream", ctypes.c_void_p),
        ("device_buffer", ctypes.c_void_p),
        ("device_buffer_bytes", ctypes.c_uint64),
    ]


class lbm_stats(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int64), ("steps", ctypes.c_int64),
        ("theta_mean", ctypes.c_double), ("theta_var", ctypes.c_double),
        ("theta_skew", ctypes.c_double), ("theta_flat", ctypes.c_double),
        ("theta_min", ctypes.c_double), ("theta_max", ctypes.c_double),
        ("kt_mean", ctypes.c_double), ("kt_var", ctypes.c_double),
        ("kt_skew", ctypes.c_double), ("kt_flat", ctypes.c_double),
        ("kt_min", ctypes.c_double), ("kt_max", ctypes.c_double),
        ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
        ("energy", ctypes.c_double), ("energy_rho", ctypes.c_double),
        ("n_nonfinite", ctypes.c_int64),
        ("strain2", ctypes.c_double), ("nut_strain2", ctypes.c_double),
        ("injection", ctypes.c_double),
        ("u_mean", ctypes.c_double * 3), ("uu", ctypes.c_double * 6),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name in ("momentum", "u_mean", "uu") else v
        return out


class lbm_turbulence_stats(ctypes.Structure):
    _fields_ = [
        ("kmax", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("energy", ctypes.c_double), ("energy_spec", ctypes.c_double),
        ("u_rms", ctypes.c_double), ("integral_scale", ctypes.c_double),
        ("eps_spec", ctypes.c_double), ("eps_strain", ctypes.c_double),
        ("eps_sgs", ctypes.c_double), ("injection", ctypes.c_double),
        ("eta", ctypes.c_double), ("taylor", ctypes.c_double), ("re_lambda", ctypes.c_double),
        ("energy_frac", ctypes.c_double * 3), ("b", ctypes.c_double * 6),
        ("II_b", ctypes.c_double), ("III_b", ctypes.c_double),
        ("lumley_xi", ctypes.c_double), ("lumley_eta", ctypes.c_double),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            if name != "pad":
                v = getattr(self, name)
                out[name] = list(v) if name in ("energy_frac", "b") else v
        return out


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load liblbm.so (raises RuntimeError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2512_23116_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lbm_config_default": (None, [ctypes.POINTER(lbm_config)]),
        "lbm_required_bytes": (ctypes.c_size_t, [ctypes.POINTER(lbm_config)]),
        "lbm_create": (ctypes.c_int, [ctypes.POINTER(lbm_config), ctypes.POINTER(H)]),
        "lbm_init_seeded": (ctypes.c_int, [H, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64]),
        "lbm_init_velocity": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_void_p]),
        "lbm_step": (ctypes.c_int, [H, ctypes.c_int64]),
        "lbm_stream_only": (ctypes.c_int, [H, ctypes.c_int64]),
        "lbm_moments": (ctypes.c_int, [H, dp, dp]),
        "lbm_kt_stats": (ctypes.c_int, [H, ctypes.POINTER(lbm_stats)]),
        "lbm_kt_field": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_float)]),
        "lbm_kt_slice": (ctypes.c_int, [H, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
        "lbm_get_populations": (ctypes.c_int, [H, dp]),
        "lbm_set_populations": (ctypes.c_int, [H, dp]),
        "lbm_sample_populations": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_int64),
                                                  ctypes.c_int64, dp]),
        "lbm_synchronize": (ctypes.c_int, [H]),
        "lbm_set_stream": (ctypes.c_int, [H, ctypes.c_void_p]),
        "lbm_theta_histogram": (ctypes.c_int, [H, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
        "lbm_theta_histogram_noalloc": (ctypes.c_int, [H, ctypes.c_double, ctypes.c_double,
                                                       ctypes.c_int32,
                                                       ctypes.POINTER(ctypes.c_int64)]),
        "lbm_spectrum": (ctypes.c_int, [H, ctypes.c_int32, dp]),
        "lbm_snapshot_begin": (ctypes.c_int, [H, ctypes.c_int32, ctypes.c_int32]),
        "lbm_snapshot_end": (ctypes.c_int, [H, ctypes.POINTER(lbm_stats), dp,
                                            ctypes.POINTER(ctypes.c_float)]),
        "lbm_spectra_1d": (ctypes.c_int, [H, ctypes.c_int32, dp, dp]),
        "lbm_structure_functions": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_int32),
                                                   ctypes.c_int32, dp]),
        "lbm_turbulence": (ctypes.c_int, [H, ctypes.c_int32,
                                          ctypes.POINTER(lbm_turbulence_stats)]),
        "lbm_state_bytes": (ctypes.c_size_t, [H]),
        "lbm_save_state": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_int64)]),
        "lbm_load_state": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64]),
        "lbm_steps_done": (ctypes.c_int64, [H]),
        "lbm_num_cells": (ctypes.c_int64, [H]),
        "lbm_destroy": (None, [H]),
        "lbm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lbm_last_error": (ctypes.c_char_p, [H]),
        "lbm_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(H)]),
        "lbm_batch_step": (ctypes.c_int, [H, ctypes.POINTER(H), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.c_int32]),
        "lbm_batch_last_error": (ctypes.c_char_p, [H]),
        "lbm_batch_destroy": (None, [H]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status, handle=None, batch=None):
    if status != LBM_OK:
        L = lib()
        if batch is not None:
            msg = L.lbm_batch_last_error(batch)
        else:
            msg = L.lbm_last_error(handle)
        raise LbmError(status, (msg or b"").decode() or L.lbm_status_string(status).decode())


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------- C names ---

def lbm_config_default():
    cfg = lbm_config()
    lib().lbm_config_default(ctypes.byref(cfg))
    return cfg


def lbm_required_bytes(cfg):
    return int(lib().lbm_required_bytes(ctypes.byref(cfg)))


def lbm_create(cfg):
    h = ctypes.c_void_p()
    _check(lib().lbm_create(ctypes.byref(cfg), ctypes.byref(h)), None)
    return h


def lbm_init_seeded(h, kind, amplitude, seed):
    _check(lib().lbm_init_seeded(h, kind, amplitude, seed & ((1 << 64) - 1)), h)


def lbm_init_velocity(h, u_ptr, rho_ptr=None):
    """u_ptr, rho_ptr: device addresses (int) of FP64 arrays, rho_ptr may be None."""
    _check(lib().lbm_init_velocity(h, ctypes.c_void_p(u_ptr),
                                   None if rho_ptr is None else ctypes.c_void_p(rho_ptr)), h)


def lbm_step(h, n):
    _check(lib().lbm_step(h, n), h)


def lbm_stream_only(h, n):
    _check(lib().lbm_stream_only(h, n), h)


def lbm_moments(h, ncell):
    rho = np.empty(ncell)
    u = np.empty(3 * ncell)
    _check(lib().lbm_moments(h, _dp(rho), _dp(u)), h)
    return rho, u.reshape(3, ncell)


def lbm_kt_stats(h, allow_unstable=False):
    st = lbm_stats()
    rc = lib().lbm_kt_stats(h, ctypes.byref(st))
    if not (allow_unstable and rc == LBM_ERR_UNSTABLE):
        _check(rc, h)
    return st.as_dict()


def lbm_kt_field(h, ncell, out=None):
    """K_t per cell into `out` (C-contiguous float32 with ncell elements; a
    page-locked buffer makes the copy one DMA) or into a new array."""
    if out is None:
        kt = np.empty(ncell, dtype=np.float32)
    else:
        if out.dtype != np.float32 or out.size != ncell or not out.flags.c_contiguous \
                or not out.flags.writeable:
            raise ValueError("out must be a writeable C-contiguous float32 array of ncell elements")
        kt = out.reshape(-1)
    _check(lib().lbm_kt_field(h, kt.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), h)
    return kt


def lbm_kt_slice(h, z, nxy):
    kt = np.empty(nxy, dtype=np.float32)
    _check(lib().lbm_kt_slice(h, z, kt.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), h)
    return kt


def lbm_get_populations(h, ncell):
    f = np.empty(19 * ncell)
    _check(lib().lbm_get_populations(h, _dp(f)), h)
    return f.reshape(19, ncell)


def lbm_set_populations(h, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(lib().lbm_set_populations(h, _dp(f)), h)


def lbm_sample_populations(h, cells):
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((len(cells), 19))
    _check(lib().lbm_sample_populations(
        h, cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(cells), _dp(out)), h)
    return out


def lbm_save_state(h):
    n = int(lib().lbm_state_bytes(h))
    buf = np.empty(n, dtype=np.uint8)
    steps = ctypes.c_int64()
    _check(lib().lbm_save_state(h, buf.ctypes.data, n, ctypes.byref(steps)), h)
    return buf, steps.value


def lbm_load_state(h, buf, steps):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().lbm_load_state(h, buf.ctypes.data, buf.size, steps), h)


def lbm_theta_histogram(h, lo, hi, nbins):
    counts = np.empty(nbins + 3, dtype=np.int64)
    _check(lib().lbm_theta_histogram(h, lo, hi, nbins,
                                     counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), h)
    return counts


def lbm_theta_histogram_noalloc(h, lo, hi, nbins):
    counts = np.empty(nbins + 3, dtype=np.int64)
    _check(lib().lbm_theta_histogram_noalloc(
        h, lo, hi, nbins, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), h)
    return counts


def lbm_spectrum(h, kmax):
    E = np.empty(kmax + 1)
    _check(lib().lbm_spectrum(h, kmax, _dp(E)), h)
    return E


def lbm_snapshot_begin(h, kmax, z):
    _check(lib().lbm_snapshot_begin(h, kmax, z), h)


def lbm_snapshot_end(h, kmax, nxy, allow_unstable=False):
    st = lbm_stats()
    E = np.empty(kmax + 1)
    plane = np.empty(nxy, dtype=np.float32)
    status = lib().lbm_snapshot_end(h, ctypes.byref(st), _dp(E),
                                    plane.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    if not (allow_unstable and status == LBM_ERR_UNSTABLE):
        _check(status, h)
    return st.as_dict(), E, plane


def lbm_spectra_1d(h, kmax, with_ic=True):
    """(E[c, a, k] (3, 3, kmax+1), IC[k] or None)."""
    E = np.empty((3, 3, kmax + 1))
    ic = np.empty(kmax + 1) if with_ic else None
    _check(lib().lbm_spectra_1d(h, kmax, _dp(E), _dp(ic) if with_ic else None), h)
    return E, ic


def lbm_structure_functions(h, rs):
    rs = np.ascontiguousarray(rs, dtype=np.int32)
    out = np.empty((len(rs), 6))
    _check(lib().lbm_structure_functions(
        h, rs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(rs), _dp(out)), h)
    return out


def lbm_turbulence(h, kmax=0):
    out = lbm_turbulence_stats()
    _check(lib().lbm_turbulence(h, int(kmax), ctypes.byref(out)), h)
    return out.as_dict()


def lbm_synchronize(h):
    _check(lib().lbm_synchronize(h), h)


def lbm_set_stream(h, stream_ptr):
    _check(lib().lbm_set_stream(h, stream_ptr), h)


def lbm_steps_done(h):
    return int(lib().lbm_steps_done(h))


def lbm_destroy(h):
    lib().lbm_destroy(h)


def lbm_batch_create(max_slots, steps_per_graph, stream):
    b = ctypes.c_void_p()
    _check(lib().lbm_batch_create(max_slots, steps_per_graph, stream, ctypes.byref(b)), None)
    return b


def lbm_batch_step(b, handles, steps):
    n = len(handles)
    arr = (ctypes.c_void_p * max(n, 1))(*[h.value for h in handles])
    st = (ctypes.c_int32 * max(n, 1))(*steps)
    _check(lib().lbm_batch_step(b, arr, st, n), batch=b)


def lbm_batch_destroy(b):
    lib().lbm_batch_destroy(b)


# ------------------------------------------------------- convenience ---

def make_modes(modes):
    """ctypes array of lbm_force_mode from ``(k, amp, phase)`` tuples."""
    arr = (lbm_force_mode * max(len(modes), 1))()
    for i, (k, amp, phase) in enumerate(modes):
        arr[i].k[:] = [int(v) for v in k]
        arr[i].reserved = 0
        arr[i].amp[:] = [float(v) for v in amp]
        arr[i].phase = float(phase)
    return arr


class Lattice:
    """One lattice on the current HIP device: owns its handle and torch buffer.

    shape is (nz, ny, nx); modes are (k, amp, phase) triples of the body force;
    precision "fp64" | "fp32" | "fp16" | "bf16"; streaming "aa" | "ab".  Arrays
    come back as (…, nz, ny, nx) with x fastest, the canonical pre-collision
    state after `steps` steps.  Every method is one C-ABI call (include/lbm.h).
    """

    def __init__(self, shape, tau0, C, modes=(), precision="fp32", streaming="aa",
                 smag_form=0, steps_per_graph=64, storage_scale=0.0, stream=None, rho0=1.0,
                 temporal_block=0, tau_mode=0):
        import torch
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.ncell = nx * ny * nz
        cfg = lbm_config_default()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.precision = PRECISION[precision] if isinstance(precision, str) else precision
        cfg.streaming = STREAMING[streaming] if isinstance(streaming, str) else streaming
        cfg.smag_form = smag_form
        cfg.tau0 = tau0
        cfg.smag_C = C
        cfg.rho0 = rho0
        cfg.storage_scale = storage_scale
        cfg.steps_per_graph = steps_per_graph
        cfg.temporal_block = temporal_block
        cfg.tau_mode = tau_mode
        self._modes = make_modes(list(modes))
        cfg.n_force_modes = len(modes)
        cfg.force_modes = ctypes.cast(self._modes, ctypes.POINTER(lbm_force_mode))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        cfg.hip_stream = stream.cuda_stream
        nbytes = lbm_required_bytes(cfg)
        if nbytes == 0:
            # invalid config: let lbm_create report why
            cfg.device_buffer = None
            self.handle = lbm_create(cfg)
        with torch.cuda.stream(stream):
            self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        ptr = self.buffer.data_ptr()
        cfg.device_buffer = (ptr + 255) // 256 * 256
        cfg.device_buffer_bytes = nbytes
        self.cfg = cfg
        self.handle = lbm_create(cfg)

    def init(self, kind, amp, seed=0):
        """lbm_init_seeded: equilibrium of an LBM_INIT_* velocity field; steps = 0."""
        lbm_init_seeded(self.handle, kind, amp, seed)
        return self

    def init_velocity(self, u, rho=None):
        """lbm_init_velocity: equilibrium of a velocity (and density) field held in
        torch CUDA float64 tensors of shape (3, nz, ny, nx) (and (nz, ny, nx));
        steps = 0.  Ordered after the work queued on torch's current stream, and
        waits for the lattice's stream before it returns, so the tensors may be
        freed afterwards."""
        import torch
        nz, ny, nx = self.shape
        if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64
                and tuple(u.shape) == (3, nz, ny, nx)):
            raise ValueError("u must be a CUDA float64 tensor of shape (3, nz, ny, nx)")
        if rho is not None and not (isinstance(rho, torch.Tensor) and rho.is_cuda
                                    and rho.dtype == torch.float64
                                    and tuple(rho.shape) == (nz, ny, nx)):
            raise ValueError("rho must be a CUDA float64 tensor of shape (nz, ny, nx)")
        u = u.contiguous()
        rho = None if rho is None else rho.contiguous()
        self.stream.wait_stream(torch.cuda.current_stream())
        lbm_init_velocity(self.handle, u.data_ptr(), None if rho is None else rho.data_ptr())
        self.sync()
        return self

    def step(self, n=1):
        """lbm_step: n time steps, asynchronous on the lattice's stream."""
        lbm_step(self.handle, n)
        return self

    def stream_only(self, n=1):
        """lbm_stream_only: n steps of free streaming (the step's data movement,
        no collision), asynchronous."""
        lbm_stream_only(self.handle, n)
        return self

    def sync(self):
        """lbm_synchronize: wait for the lattice's stream."""
        lbm_synchronize(self.handle)

    def set_stream(self, stream):
        """lbm_set_stream: later calls run on `stream` (a torch.cuda.Stream).  The
        caller orders it after the work pending on the old stream."""
        lbm_set_stream(self.handle, stream.cuda_stream)
        self.stream = stream

    @property
    def steps(self):
        """Time steps done since the last init / load."""
        return lbm_steps_done(self.handle)

    def populations(self):
        """lbm_get_populations: full f, (19, nz, ny, nx) FP64."""
        return lbm_get_populations(self.handle, self.ncell).reshape((19,) + self.shape)

    def set_populations(self, f):
        """lbm_set_populations: replace the state by full f, (19, ...) FP64."""
        lbm_set_populations(self.handle, np.asarray(f).reshape(19, -1))

    def moments(self):
        """lbm_moments: rho (nz, ny, nx) and the Guo velocity u (3, nz, ny, nx)."""
        rho, u = lbm_moments(self.handle, self.ncell)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape)

    def stats(self, allow_unstable=False):
        """lbm_kt_stats: dict of the FP64 theta / K_t statistics, mass, momentum,
        energy and the energy-balance sums; raises on a non-finite state unless
        allow_unstable."""
        return lbm_kt_stats(self.handle, allow_unstable)

    def kt_field(self, out=None):
        """lbm_kt_field: K_t per cell, (nz, ny, nx) float32 (into `out` if given)."""
        return lbm_kt_field(self.handle, self.ncell, out).reshape(self.shape)

    def theta_histogram(self, lo, hi, nbins):
        """lbm_theta_histogram: int64[nbins + 3] = [below lo, bins..., at or above
        hi, non-finite]."""
        return lbm_theta_histogram(self.handle, lo, hi, nbins)

    def theta_histogram_noalloc(self, lo, hi, nbins):
        """lbm_theta_histogram_noalloc: the same counts from the library's static
        device scratch (no device allocation; nbins <= 4096)."""
        return lbm_theta_histogram_noalloc(self.handle, lo, hi, nbins)

    def kt_slice(self, z):
        """K_t of plane z as an (ny, nx) array."""
        return lbm_kt_slice(self.handle, z, self.shape[1] * self.shape[2]).reshape(self.shape[1:])

    def spectrum(self, kmax):
        """lbm_spectrum: shell spectrum E(0..kmax)."""
        return lbm_spectrum(self.handle, kmax)

    def snapshot_begin(self, kmax, z):
        """lbm_snapshot_begin: enqueue the statistics, the K_t map of plane z and the
        spectrum E(0..kmax) of the current state; returns at once."""
        lbm_snapshot_begin(self.handle, kmax, z)
        self._snap_kmax = kmax

    def snapshot_end(self, allow_unstable=False):
        """lbm_snapshot_end: (stats dict, E[0..kmax], K_t plane (ny, nx)) of the
        snapshot begun last."""
        st, E, plane = lbm_snapshot_end(self.handle, self._snap_kmax,
                                        self.shape[1] * self.shape[2], allow_unstable)
        return st, E, plane.reshape(self.shape[1:])

    def spectra_1d(self, kmax, with_ic=True):
        """lbm_spectra_1d: (E[c, a, k] of shape (3, 3, kmax+1), IC(k) or None)."""
        return lbm_spectra_1d(self.handle, kmax, with_ic)

    def structure_functions(self, rs):
        """lbm_structure_functions: (len(rs), 6) moments of longitudinal increments."""
        return lbm_structure_functions(self.handle, rs)

    def turbulence(self, kmax=0):
        """lbm_turbulence: dict of the turbulence scales and isotropy measures."""
        return lbm_turbulence(self.handle, kmax)

    def save(self):
        """lbm_save_state: (state bytes as uint8 array, steps)."""
        return lbm_save_state(self.handle)

    def load(self, buf, steps):
        """lbm_load_state: restore a saved state and its step count."""
        lbm_load_state(self.handle, buf, steps)

    def sample(self, cells):
        """lbm_sample_populations: full f of the listed cell indices, (n, 19)."""
        return lbm_sample_populations(self.handle, cells)

    def close(self):
        """lbm_destroy; also drops the torch buffer.  Safe to call twice."""
        if getattr(self, "handle", None) is not None and self.handle.value:
            lbm_destroy(self.handle)
            self.handle = None
        self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
