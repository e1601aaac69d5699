"""Initial velocity fields and the equilibrium start (oracle side).

Test infrastructure only (see ``oracle/__init__.py``).

Reading (the paper names Taylor-Green vortices after Brachet et al. but
prints no formula, Sec. 2.2 and Sec. 3.1): the 3-D field is
u = A sin X cos Y cos Z, v = -A cos X sin Y cos Z, w = 0 with
X = 2 pi x/nx, Y = 2 pi y/ny, Z = 2 pi z/nz.  The initial populations are the
second-order equilibrium of App. A eq. feq at rho = rho0 = 1 and that velocity,
without any half-force shift.

The seeded noise start (zero-mean velocity noise of amplitude A) is not in the
paper; it uses SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based
hash, implemented here from its published definition:
  U(cell, a) = (splitmix64(splitmix64(seed) XOR (3*cell + a)) >> 11) * 2^-53,
  u_a = A (2 U - 1), cell = x + nx (y + ny z).
"""
import numpy as np

from .ref_numpy import feq

KIND_NOISE, KIND_TGV3D, KIND_TGV2D, KIND_SHEAR, KIND_REST = 0, 1, 2, 3, 4

_MASK = (1 << 64) - 1


def splitmix64(v):
    """One SplitMix64 output for state ``v`` (Python ints, exact 64-bit arithmetic)."""
    z = (v + 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def _splitmix64_array(v):
    """Vectorised SplitMix64 over a uint64 array (numpy wraps modulo 2^64)."""
    z = v + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def noise_uniform(shape, seed):
    """U in [0, 1) per cell and component: array (3, nz, ny, nx)."""
    nz, ny, nx = shape
    key = np.uint64(splitmix64(seed & _MASK))
    cell = np.arange(nx * ny * nz, dtype=np.uint64)
    out = np.empty((3, nx * ny * nz))
    with np.errstate(over="ignore"):
        for a in range(3):
            h = _splitmix64_array(key ^ (np.uint64(3) * cell + np.uint64(a)))
            out[a] = (h >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return out.reshape((3, nz, ny, nx))


def velocity(kind, shape, amp, seed=0):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X, Y, Z = 2 * np.pi * x / nx, 2 * np.pi * y / ny, 2 * np.pi * z / nz
    u = np.zeros((3,) + tuple(shape))
    if kind == KIND_TGV3D:
        u[0] = amp * np.sin(X) * np.cos(Y) * np.cos(Z)
        u[1] = -amp * np.cos(X) * np.sin(Y) * np.cos(Z)
    elif kind == KIND_TGV2D:
        u[0] = amp * np.sin(X) * np.cos(Y)
        u[1] = -amp * np.cos(X) * np.sin(Y)
    elif kind == KIND_SHEAR:
        u[0] = amp * np.sin(Y)
    elif kind == KIND_NOISE:
        u = amp * (2.0 * noise_uniform(shape, seed) - 1.0)
    elif kind != KIND_REST:
        raise ValueError(f"unknown init kind {kind}")
    return u


def initial_populations(kind, shape, amp, seed=0, rho0=1.0):
    """f(x, 0) = f^eq(rho0, u0(x)) (App. A eq. feq), full populations (19, nz, ny, nx)."""
    u = velocity(kind, shape, amp, seed)
    rho = np.full(tuple(shape), rho0)
    return feq(rho, u)
