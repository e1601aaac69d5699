"""Parameter relations of the paper (oracle side; test infrastructure only).

All quantities in lattice units, delta_x = delta_t = 1, c_s^2 = 1/3 (App. A).
"""
import math

CS2 = 1.0 / 3.0


def nu_from_tau(tau):
    """nu = c_s^2 (1/s_nu - 1/2) delta_t, Sec. 2.1 eq. bare_viscosity."""
    return CS2 * (tau - 0.5)


def tau_from_nu(nu):
    return 0.5 + nu / CS2


def reynolds(U0, N, nu0):
    """Re = U0 N_x / nu0, Sec. 3.1."""
    return U0 * N / nu0


def tau0_from_re(U0, N, Re):
    """tau0 = 1/2 + 3 U0 N / Re (Sec. 3.1 with eq. bare_viscosity)."""
    return tau_from_nu(U0 * N / Re)


def forcing_amplitude(U0, N, C_f=0.2, rho=1.0):
    """F0 = C_f rho U0^2 / N_x, Sec. 2.2 eq. forcing_amplitude."""
    return C_f * rho * U0 * U0 / N


def k41_strain(U0, L, ell=1.0):
    """|S| ~ U0 / (L^(1/3) ell^(2/3)), the K41 estimate of Sec. 4."""
    return U0 / (L ** (1.0 / 3.0) * ell ** (2.0 / 3.0))


def turbulent_tau(C, S, Delta=1.0):
    """tau_t = C Delta^2 |S| / c_s^2, Sec. 4."""
    return C * Delta * Delta / CS2 * S


def tau_offset(U0, N, Re, C, S, Delta=1.0):
    """tau_e - 1/2 = 3 (U0 N/Re + C Delta^2 |S|), Sec. 2.3 eq. tau_offset_scaling."""
    return 3.0 * (U0 * N / Re + C * Delta * Delta * S)


def knudsen_turbulent(theta, ell=1.0, dx=1.0):
    """K_t = (tau_e - 1/2) sqrt(3) delta_x / ell, Sec. 2.4 eq. Kt_definition."""
    return theta * math.sqrt(3.0) * dx / ell
