"""Pope's model spectrum, the reference the paper holds its DNS spectra against
(Sec. 3.4, eq. pope_model, Fig. DNS_spectra_validation).

The paper prints E(k) = C_K eps^(2/3) k^(-5/3) f_L(kL) f_eta(k eta) with C_K = 1.5
and refers to Pope (Turbulent Flows, 2000, Sec. 6.5.3) for the two shape
functions; this module restates that published model:

    f_L(kL)       = (kL / ((kL)^2 + c_L)^(1/2))^(5/3 + p0),        p0 = 2,
    f_eta(k eta)  = exp(-beta (((k eta)^4 + c_eta^4)^(1/4) - c_eta)),  beta = 5.2,

with L = k_t^(3/2) / eps (k_t the turbulent kinetic energy) and c_L, c_eta the
two constants that make the model carry the measured k_t and eps:
integral of E = k_t and 2 nu * integral of k^2 E = eps.  (Only (L/eta)^2 / c_L
enters f_L, so any other choice of L changes c_L and nothing else.)  At high
Reynolds number this gives Pope's c_L = 6.78, c_eta = 0.40.

Everything is in Kolmogorov units: x = kappa eta, E / (eps nu^5)^(1/4); there
the constraints read  integral E dx = k_t / (eps nu)^(1/2)  and
2 integral x^2 E dx = 1, and L / eta = (k_t / (eps nu)^(1/2))^(3/2).

Host-side post-processing of a spectrum the device has measured.
"""
import numpy as np

C_K, P0, BETA = 1.5, 2.0, 5.2
_X = np.geomspace(1e-10, 60.0, 40000)      # integration grid in x = kappa eta


def model(x, L_over_eta, c_L, c_eta):
    """Pope's E(kappa) / (eps nu^5)^(1/4) at x = kappa eta."""
    x = np.asarray(x, dtype=np.float64)
    y = x * L_over_eta
    f_L = (y / np.sqrt(y * y + c_L)) ** (5.0 / 3.0 + P0)
    f_eta = np.exp(-BETA * ((x ** 4 + c_eta ** 4) ** 0.25 - c_eta))
    return C_K * x ** (-5.0 / 3.0) * f_L * f_eta


def constants(K):
    """(c_L, c_eta, L / eta) for the turbulent kinetic energy K = k_t / (eps nu)^(1/2)
    in Kolmogorov units, from the energy and dissipation constraints."""
    from scipy.optimize import fsolve
    L_over_eta = K ** 1.5

    def residual(p):
        m = model(_X, L_over_eta, p[0], p[1])
        return [np.trapezoid(m, _X) / K - 1.0, 2.0 * np.trapezoid(_X * _X * m, _X) - 1.0]

    sol, _, ier, msg = fsolve(residual, [6.78, 0.40], full_output=True)
    if ier != 1 or sol[0] <= 0.0 or sol[1] <= 0.0:
        raise RuntimeError(f"Pope constants did not converge for K = {K}: {msg}")
    return float(sol[0]), float(sol[1]), float(L_over_eta)


def compare(k_eta, E_kolmogorov, band=(0.05, 1.0)):
    """Measured shell spectrum in Kolmogorov units (shells k = 1, 2, ... at
    x_k = k x_1) against Pope's model carrying the same energy and dissipation.

    K is the measured energy, sum_k E(x_k) x_1 (the shell width in x).  Returns
    the constants, the model on the measured grid, and the mean and largest
    |ln(E / E_model)| over the shells with band[0] <= x <= band[1]."""
    x = np.asarray(k_eta, dtype=np.float64)
    E = np.asarray(E_kolmogorov, dtype=np.float64)
    K = float(E.sum() * x[0])
    try:
        c_L, c_eta, L_over_eta = constants(K)
    except RuntimeError as e:           # e.g. too little energy for the model's shape
        return dict(K=K, converged=False, error=str(e))
    Em = model(x, L_over_eta, c_L, c_eta)
    sel = (x >= band[0]) & (x <= band[1]) & (E > 0)
    lr = np.abs(np.log(E[sel] / Em[sel])) if sel.any() else np.array([np.nan])
    return dict(K=K, converged=True, c_L=c_L, c_eta=c_eta, L_over_eta=L_over_eta,
                E_model=[float(v) for v in Em], band=list(band), shells_in_band=int(sel.sum()),
                mean_abs_log_ratio=float(lr.mean()), max_abs_log_ratio=float(lr.max()))
