"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds none of the method's arithmetic: it only draws and lays out
the forcing-mode tables that both sides receive as inputs.  The random numbers
come from numpy's PCG64 generator with an explicit seed.

A forcing mode is ``(k, amp, phase)``: integer wavevector k = (kx, ky, kz),
amplitude vector amp (3,), phase in radians.  The body force is the sum over
modes of amp * sin(2 pi (kx x/nx + ky y/ny + kz z/nz) + phase).
"""
import math

import numpy as np


def paper_modes(F0):
    """The paper's stationary three-mode pattern (Sec. 2.2, eq. forcing_pattern).

    F_x = F0 sin(2 pi y/N), F_y = F0 sin(2 pi z/N), F_z = F0 sin(2 pi x/N).
    """
    return [((0, 1, 0), (F0, 0.0, 0.0), 0.0),
            ((0, 0, 1), (0.0, F0, 0.0), 0.0),
            ((1, 0, 0), (0.0, 0.0, F0), 0.0)]


def shell_wavevectors(kmax2=4):
    """One representative of each +-k pair with 1 <= |k|^2 <= kmax2, fixed order.

    The representative is the one whose first non-zero component is positive.
    For kmax2 = 4 there are 16 of them (3 + 6 + 4 + 3 by |k|^2 = 1, 2, 3, 4).
    """
    r = int(math.isqrt(kmax2))
    out = []
    for k2 in range(1, kmax2 + 1):
        for kx in range(-r, r + 1):
            for ky in range(-r, r + 1):
                for kz in range(-r, r + 1):
                    if kx * kx + ky * ky + kz * kz != k2:
                        continue
                    first = next(c for c in (kx, ky, kz) if c != 0)
                    if first > 0:
                        out.append((kx, ky, kz))
    return out


def random_solenoidal_modes(F0, seed, kmax2=4):
    """Large-scale forcing on all shells 1 <= |k|^2 <= kmax2 with seeded phases.

    Each mode gets a unit polarisation perpendicular to k (so the force is
    divergence-free) at a uniformly drawn angle, and a uniformly drawn phase.
    All modes share one amplitude A chosen so that the domain mean of |F|^2
    equals that of the three-mode pattern, 3 F0^2 / 2:  n_modes A^2 / 2 =
    3 F0^2 / 2.
    """
    ks = shell_wavevectors(kmax2)
    rng = np.random.Generator(np.random.PCG64(seed))
    A = F0 * math.sqrt(3.0 / len(ks))
    modes = []
    for k in ks:
        kv = np.array(k, dtype=np.float64)
        kh = kv / np.linalg.norm(kv)
        # orthonormal basis (e1, e2) of the plane perpendicular to k
        helper = np.array([1.0, 0.0, 0.0]) if abs(kh[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(kh, helper)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(kh, e1)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        phase = rng.uniform(0.0, 2.0 * math.pi)
        amp = A * (math.cos(ang) * e1 + math.sin(ang) * e2)
        modes.append((k, tuple(float(a) for a in amp), float(phase)))
    return modes


def serving_requests(n, seed, sizes=(32, 48, 64, 96, 128), C_range=(0.08, 0.18),
                     tau_range=(0.505, 0.55), rate=None):
    """A seeded stream of independent LES requests.

    Returns a list of dicts with N, C, tau0, forcing seed, init seed and the
    arrival time (Poisson process of the given rate; all at t = 0 if None).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n):
        if rate is not None:
            t += rng.exponential(1.0 / rate)
        out.append(dict(
            rid=i,
            N=int(rng.choice(sizes)),
            C=float(rng.uniform(*C_range)),
            tau0=float(rng.uniform(*tau_range)),
            force_seed=int(rng.integers(0, 2 ** 31)),
            init_seed=int(rng.integers(0, 2 ** 31)),
            arrival=t,
        ))
    return out
