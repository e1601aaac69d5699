"""Dense literal definition of the LBM-MRT-Smagorinsky-Guo time step (FP64).

Test infrastructure only (see ``oracle/__init__.py``).  Slow on purpose: dense
19x19 products, ``np.linalg.inv(M)`` and ``np.roll`` streaming, meant for brute
force on lattices up to ~16^3.

Arrays: populations ``f`` have shape (19, nz, ny, nx) (x fastest); vector
fields have shape (3, nz, ny, nx) with components (x, y, z).  Cell
coordinates are 0-based, ``(x, y, z) = (i, j, k)`` of the paper's forcing
formula (reading: the paper's 1-based Fortran indices shift the lattice by one
cell, which changes no statistic).

Readings of the paper used here (each is also listed in the design notes):
* The printed m^eq (App. B, eq. meq_fm) is the equilibrium of the deviation
  populations f - w rho0: its row 0 is delta-rho.  With full populations the
  rest-state moments M w rho0 = rho0 (1, -11, 3, 0, ..., 0) are added back.
* eq. yu_strain uses s_1 = 1.19 and s_9 = 1/tau0 (the bare shear rate), so
  tau_e follows from printed formulas without iteration (``tau_mode=0``).  The
  alternative ``tau_mode=1`` makes it self-consistent: s_9 = 1/tau_e and the
  divergence (m_1) term dropped, solved in closed form (``effective_tau_sc``).
* nu_t = C Delta^2 |S| with the model constant C entering linearly
  (eq. eddy_visc); ``smag_form=1`` squares it (C_s^2 convention).
* Delta = delta_x = delta_t = rho0 = 1 (App. A; App. B.1).
"""
import numpy as np

from . import d3q19 as L


def force_field(shape, modes):
    """Body force F(x) = sum_m a_m sin(2 pi k_m . (x/nx, y/ny, z/nz) + phi_m).

    The paper's pattern (Sec. 2.2, eq. forcing_pattern) is the three-mode
    instance F_x = F0 sin(2 pi y/N), F_y = F0 sin(2 pi z/N),
    F_z = F0 sin(2 pi x/N) with zero phases.  ``modes`` is a sequence of
    ``(k, amp, phase)`` with integer k (3,), amp (3,).
    """
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    F = np.zeros((3,) + tuple(shape))
    for k, amp, phase in modes:
        arg = 2 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + phase
        s = np.sin(arg)
        for a in range(3):
            F[a] += amp[a] * s
    return F


def feq(rho, u):
    """Second-order equilibrium, App. A eq. feq (c_s^2 = 1/3)."""
    cu = np.tensordot(L.C.astype(np.float64), u, axes=([1], [0]))   # (19, ...)
    uu = (u * u).sum(0)
    return L.W.reshape((19,) + (1,) * rho.ndim) * rho * (
        1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)


def guo_source(u, F):
    """Guo discrete source Phi_alpha, App. A eq. guo_force (c_s^2 = 1/3)."""
    c = L.C.astype(np.float64)
    cu = np.tensordot(c, u, axes=([1], [0]))                        # (19, ...)
    out = np.zeros((19,) + u.shape[1:])
    for a in range(19):
        vec = 3 * (c[a].reshape((3,) + (1,) * (u.ndim - 1)) - u) \
            + 9 * cu[a] * c[a].reshape((3,) + (1,) * (u.ndim - 1))
        out[a] = L.W[a] * (vec * F).sum(0)
    return out


def macroscopic(f, F):
    """rho = sum f, rho u = sum f c + F/2 (App. A eq. guo_velocity, eq. macroscopic_eq)."""
    rho = f.sum(0)
    j = np.tensordot(L.C.T.astype(np.float64), f, axes=([1], [0]))
    u = (j + 0.5 * F) / rho
    return rho, u


def equilibrium_moments(rho, u, rho0=1.0):
    """m^eq of App. B eq. meq_fm, plus the rest-state offset rho0*(1,-11,3,0,...)."""
    ux, uy, uz = u
    u2 = ux * ux + uy * uy + uz * uz
    drho = rho - rho0
    z = np.zeros_like(rho)
    meq = np.stack([
        drho,
        -11 * drho + 19 * rho * u2,
        -475.0 / 63.0 * rho * u2,
        rho * ux, -2 * rho * ux / 3,
        rho * uy, -2 * rho * uy / 3,
        rho * uz, -2 * rho * uz / 3,
        rho * (2 * ux * ux - uy * uy - uz * uz),
        z,
        rho * (uy * uy - uz * uz),
        z,
        rho * ux * uy, rho * uy * uz, rho * ux * uz,
        z, z, z,
    ])
    offset = rho0 * np.array([1.0, -11.0, 3.0] + [0.0] * 16)
    return meq + offset.reshape((19,) + (1,) * rho.ndim)


def force_moments(u, F):
    """F_m of App. B eq. meq_fm."""
    ux, uy, uz = u
    Fx, Fy, Fz = F
    uF = ux * Fx + uy * Fy + uz * Fz
    z = np.zeros_like(ux)
    return np.stack([
        z,
        38 * uF, -11 * uF,
        Fx, -2 * Fx / 3, Fy, -2 * Fy / 3, Fz, -2 * Fz / 3,
        2 * (2 * ux * Fx - uy * Fy - uz * Fz),
        -(2 * ux * Fx - uy * Fy - uz * Fz),
        2 * (uy * Fy - uz * Fz),
        -(uy * Fy - uz * Fz),
        ux * Fy + uy * Fx, uy * Fz + uz * Fy, ux * Fz + uz * Fx,
        z, z, z,
    ])


def strain_tensor(mneq, s1, s9, rho0=1.0, dt=1.0):
    """S_ab from non-equilibrium moments, App. B.1 eq. yu_strain.

    Returns (Sxx, Syy, Szz, Sxy, Sxz, Syz).
    """
    m1, m9, m11 = mneq[1], mneq[9], mneq[11]
    m13, m14, m15 = mneq[13], mneq[14], mneq[15]
    Sxx = -(s1 * m1 + 19 * s9 * m9) / (38 * rho0 * dt)
    Syy = -(2 * s1 * m1 - 19 * s9 * (m9 - 3 * m11)) / (76 * rho0 * dt)
    Szz = -(2 * s1 * m1 - 19 * s9 * (m9 + 3 * m11)) / (76 * rho0 * dt)
    Sxy = -3 * s9 / (2 * rho0 * dt) * m13
    Sxz = -3 * s9 / (2 * rho0 * dt) * m15
    Syz = -3 * s9 / (2 * rho0 * dt) * m14
    return Sxx, Syy, Szz, Sxy, Sxz, Syz


def strain_norm(S):
    """|S| = sqrt(2 (Sxx^2+Syy^2+Szz^2 + 2Sxy^2 + 2Sxz^2 + 2Syz^2)), eq. strain_norm."""
    Sxx, Syy, Szz, Sxy, Sxz, Syz = S
    return np.sqrt(2 * (Sxx ** 2 + Syy ** 2 + Szz ** 2
                        + 2 * Sxy ** 2 + 2 * Sxz ** 2 + 2 * Syz ** 2))


def effective_tau(tau0, C, Snorm, smag_form=0, Delta=1.0):
    """tau_e = 1/2 + 3 (nu0 + nu_t), nu0 = (tau0 - 1/2)/3, nu_t = C Delta^2 |S|.

    Sec. 2.1 eq. bare_viscosity and Sec. 2.3 eq. nu_eff_mrt, eq. eddy_visc,
    eq. les_viscosity (c_s^2 = 1/3, delta_t = 1).
    """
    nu0 = (tau0 - 0.5) / 3.0
    Cm = C if smag_form == 0 else C * C
    nu_t = Cm * Delta ** 2 * Snorm
    return 0.5 + 3.0 * (nu0 + nu_t)


def effective_tau_sc(tau0, C, mneq, smag_form=0, rho0=1.0, Delta=1.0):
    """Self-consistent tau_e (reading of Sec. 2.3 / App. B.1 with s_9 = 1/tau_e).

    With the m_1 term of eq. yu_strain dropped, S is linear in s_9:
    S(s_9) = s_9 S_1, S_1 = eq. yu_strain at s_1 = 0, s_9 = 1.  Then
    tau_e = tau0 + 3 C Delta^2 |S_1| / tau_e, a quadratic whose positive root is
    tau_e = (tau0 + sqrt(tau0^2 + 12 C Delta^2 |S_1|)) / 2.
    """
    S1 = strain_norm(strain_tensor(mneq, s1=0.0, s9=1.0, rho0=rho0))
    Cm = C if smag_form == 0 else C * C
    return 0.5 * (tau0 + np.sqrt(tau0 * tau0 + 12.0 * Cm * Delta ** 2 * S1))


def collide(f, F, tau0, C, smag_form=0, rho0=1.0,
            s_e=L.S_E, s_eps=L.S_EPS, s_q=L.S_Q, s_pi=L.S_PI, s_m=L.S_M, tau_mode=0):
    """Post-collision populations of eq. mrt_les_guo, per cell, in the paper's order.

    f: (19, ...) full populations, F: (3, ...) body force.  tau_mode 0: s_9 = 1/tau0
    in eq. yu_strain; 1: self-consistent s_9 = 1/tau_e (``effective_tau_sc``).
    Returns (f_star, info) with info = dict(rho, u, tau_e, Snorm).
    """
    rho, u = macroscopic(f, F)
    m = np.tensordot(L.M, f, axes=([1], [0]))
    meq = equilibrium_moments(rho, u, rho0)
    Fm = force_moments(u, F)
    mneq = m - meq
    if tau_mode == 0:
        S = strain_tensor(mneq, s1=s_e, s9=1.0 / tau0, rho0=rho0)
        Snorm = strain_norm(S)
        tau_e = effective_tau(tau0, C, Snorm, smag_form)
    else:
        tau_e = effective_tau_sc(tau0, C, mneq, smag_form, rho0)
        Snorm = strain_norm(strain_tensor(mneq, s1=0.0, s9=1.0 / tau_e, rho0=rho0))
    Lam = L.relaxation_diagonal(1.0 / tau_e, s_e, s_eps, s_q, s_pi, s_m)
    mstar = m - Lam * mneq + (1.0 - 0.5 * Lam) * Fm
    fstar = np.tensordot(L.MINV, mstar, axes=([1], [0]))
    return fstar, dict(rho=rho, u=u, tau_e=tau_e, Snorm=Snorm)


def stream(fstar):
    """f_a(x + c_a, t+1) = f*_a(x, t) on the periodic box (left side of eq. mrt_dns_guo)."""
    out = np.empty_like(fstar)
    for a in range(19):
        cx, cy, cz = L.C[a]
        out[a] = np.roll(fstar[a], shift=(cz, cy, cx), axis=(0, 1, 2))
    return out


def step(f, tau0, C, modes=(), smag_form=0, nsteps=1, **rates):
    """Advance full populations f (19, nz, ny, nx) by ``nsteps`` collide+stream steps."""
    F = force_field(f.shape[1:], modes)
    for _ in range(nsteps):
        fstar, _ = collide(f, F, tau0, C, smag_form, **rates)
        f = stream(fstar)
    return f


def diagnostics(f, tau0, C, modes=(), smag_form=0, **rates):
    """Per-cell rho, u, theta = tau_e - 1/2 and K_t of the state f.

    K_t = sqrt(3) (tau_e - 1/2) delta_x / ell with ell = delta_x (Sec. 2.4,
    eq. Kt_definition; ell ~ delta_x for LES).
    """
    F = force_field(f.shape[1:], modes)
    _, info = collide(f, F, tau0, C, smag_form, **rates)
    theta = info["tau_e"] - 0.5
    return dict(rho=info["rho"], u=info["u"], theta=theta, kt=np.sqrt(3.0) * theta)
