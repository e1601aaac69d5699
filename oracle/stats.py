"""Statistics of per-cell fields and the energy spectrum (oracle side).

Test infrastructure only (see ``oracle/__init__.py``).
"""
import numpy as np


def field_stats(v):
    """Two-pass FP64 statistics of a field: n, mean, var, skewness, flatness, min, max.

    var is the population variance <(v - <v>)^2>; skewness <d^3>/var^1.5 and
    flatness <d^4>/var^2 (NaN when var == 0).  These are the domain statistics
    of tau_e - 1/2 and K_t the paper reports (Sec. 5.1).
    """
    v = np.asarray(v, dtype=np.float64).ravel()
    n = v.size
    mean = v.sum() / n
    d = v - mean
    var = (d * d).sum() / n
    if var > 0:
        skew = (d ** 3).sum() / n / var ** 1.5
        flat = (d ** 4).sum() / n / var ** 2
    else:
        skew = float("nan")
        flat = float("nan")
    return dict(n=n, mean=mean, var=var, skew=skew, flat=flat, min=v.min(), max=v.max())


def energy_spectrum(u):
    """Shell-binned spectrum E(k), Sec. 2.2 eq. integral_length_scale.

    Reading: the printed sum lacks the square; E(k) = 1/2 sum |u_hat(k)|^2 over
    k - 1/2 <= |k| < k + 1/2, with u_hat = N^-3 sum_x u(x) exp(-i k.x), so that
    sum_k E(k) = 1/2 <u.u> (Parseval).  u: (3, nz, ny, nx), integer wavenumbers.
    Returns E for k = 0 .. kmax (kmax = the largest shell index present).
    """
    u = np.asarray(u, dtype=np.float64)
    _, nz, ny, nx = u.shape
    n = nx * ny * nz
    e = np.zeros((nz, ny, nx))
    for a in range(3):
        uh = np.fft.fftn(u[a]) / n
        e += 0.5 * (uh.real ** 2 + uh.imag ** 2)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = np.floor(kmag + 0.5).astype(np.int64)
    return np.bincount(shell.ravel(), weights=e.ravel())


SF_ORDERS = ("S2", "S3", "S3abs", "S4", "S5abs", "S6")


def structure_functions(u, rs):
    """Longitudinal structure functions averaged over the three axes.

    Sec. 2.2 / 5.3 use increments of the velocity component along the
    separation: du_a(x; r) = u_a(x + r e_a) - u_a(x), periodic.  Returns an
    array (len(rs), 6) of <du^2>, <du^3>, <|du|^3>, <du^4>, <|du|^5>, <du^6>,
    each averaged over all cells and the three axes.  F4(r) = S4 / S2^2.
    """
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros((len(rs), 6))
    axis_of = {0: 2, 1: 1, 2: 0}          # component x varies along array axis 2, ...
    for j, r in enumerate(rs):
        acc = np.zeros(6)
        for a in range(3):
            du = np.roll(u[a], -r, axis=axis_of[a]) - u[a]
            d2 = du * du
            acc += [d2.mean(), (d2 * du).mean(), (d2 * np.abs(du)).mean(), (d2 * d2).mean(),
                    (d2 * d2 * np.abs(du)).mean(), (d2 * d2 * d2).mean()]
        out[j] = acc / 3.0
    return out


def turbulence_scales(u, nu0, snorm=None, tau_t=None, F=None):
    """Turbulence scales of Sec. 2.2 for a velocity field u (3, N, N, N).

    Reading: the shell index k of the N-cell periodic box is the wavenumber
    kappa = 2 pi k / N in lattice units (the paper's 2 pi box maps onto N cells),
    the mean flow (k = 0) is excluded, and the viscosity is the molecular
    nu0 = (tau0 - 1/2)/3:
      L = (3 pi / 4) sum(E / kappa) / sum(E)       eq. integral_length_scale
      u_rms = sqrt(2 sum(E) / 3)                   eq. rms_velocity
      eps_spec = 2 nu0 sum(kappa^2 E)              eq. dissipation_rate
      eta = (nu0^3 / eps)^(1/4), lambda = sqrt(15 nu0 u_rms^2 / eps)
                                                   eq. kolmogorov_scale, eq. taylor_microscale
    Given the per-cell strain magnitude |S| (eq. strain_norm), tau_t = tau_e - tau0
    and the force F: eps_strain = 2 nu0 <S:S> = nu0 <|S|^2>, eps_sgs = <nu_t |S|^2>
    with nu_t = tau_t / 3, injection = <F.u> (eq. energy_balance).
    """
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[1]
    assert u.shape[1:] == (N, N, N), "a cubic lattice"
    E = energy_spectrum(u)
    k = np.arange(1, E.size)
    kap = 2.0 * np.pi * k / N
    Ek = E[1:]
    e = Ek.sum()
    out = dict(energy=0.5 * (u * u).sum(0).mean(), energy_spec=e,
               u_rms=np.sqrt(2.0 * e / 3.0),
               integral_scale=0.75 * np.pi * (Ek / kap).sum() / e,
               eps_spec=2.0 * nu0 * (kap * kap * Ek).sum())
    eps = out["eps_spec"]
    out["eta"] = (nu0 ** 3 / eps) ** 0.25
    out["taylor"] = np.sqrt(15.0 * nu0 * out["u_rms"] ** 2 / eps)
    out["re_lambda"] = out["u_rms"] * out["taylor"] / nu0
    if snorm is not None:
        s2 = np.asarray(snorm, dtype=np.float64) ** 2
        out["eps_strain"] = nu0 * s2.mean()
        if tau_t is not None:
            out["eps_sgs"] = (np.asarray(tau_t) / 3.0 * s2).mean()
    if F is not None:
        out["injection"] = (np.asarray(F) * u).sum(0).mean()
    return out


def isotropy(u):
    """Statistical isotropy of a velocity field u (3, ...) (Sec. 3.3, Fig.
    isotropy_validation, Tab. isotropy_metrics).

    Reynolds stresses of the fluctuations R_ij = <u'_i u'_j>, directional energy
    fractions R_ii / R_kk, anisotropy b_ij = R_ij / R_kk - delta_ij / 3, invariants
    II_b = -b_ij b_ji / 2 and III_b = b_ij b_jk b_ki / 3, Lumley coordinates
    xi = (III_b / 2)^(1/3) (real cube root), eta = (-II_b / 3)^(1/2).
    """
    u = np.asarray(u, dtype=np.float64).reshape(3, -1)
    up = u - u.mean(axis=1, keepdims=True)
    R = up @ up.T / up.shape[1]
    tr = np.trace(R)
    b = R / tr - np.eye(3) / 3.0
    II = -0.5 * np.trace(b @ b)
    III = np.trace(b @ b @ b) / 3.0
    return dict(energy_frac=np.diag(R) / tr,
                b=np.array([b[0, 0], b[1, 1], b[2, 2], b[0, 1], b[0, 2], b[1, 2]]),
                II_b=II, III_b=III, lumley_xi=np.cbrt(III / 2.0), lumley_eta=np.sqrt(-II / 3.0))


def one_dimensional_spectra(u):
    """One-dimensional energy spectra of each velocity component along each axis
    (App. spectral isotropy: the longitudinal and transverse spectra E_11, E_22).

    E[c, a, k] = sum of |u_hat_c(q)|^2 over the wavevectors q with |q_a| = k,
    u_hat = FFT(u) / ncells (integer wavenumbers, k = 0 .. max_a n_a // 2;
    entries beyond n_a // 2 are zero).  Parseval per axis: sum_k E[c, a, k] =
    <u_c^2>.  Axis a = 0, 1, 2 is x, y, z; u: (3, nz, ny, nx).
    """
    u = np.asarray(u, dtype=np.float64)
    _, nz, ny, nx = u.shape
    n = nx * ny * nz
    K = max(nx, ny, nz) // 2 + 1
    out = np.zeros((3, 3, K))
    array_axis = {0: 2, 1: 1, 2: 0}        # x varies along array axis 2, ...
    for c in range(3):
        uh = np.fft.fftn(u[c]) / n
        p = uh.real ** 2 + uh.imag ** 2
        for a in range(3):
            ax = array_axis[a]
            m = p.shape[ax]
            line = p.sum(axis=tuple(d for d in range(3) if d != ax))
            k = np.abs(np.fft.fftfreq(m, 1.0 / m)).round().astype(np.int64)
            out[c, a] = np.bincount(k, weights=line, minlength=K)[:K]
    return out


def isotropy_coefficient(E):
    """Spectral isotropy coefficient IC(k) from the one-dimensional spectra E[c, a, k]
    of a cubic lattice (App. spectral isotropy).

    Reading: in isotropic turbulence the transverse spectrum follows from the
    longitudinal one, E_22 = (E_11 - k dE_11/dk) / 2 (Batchelor), so
    IC(k) = (E_L - k dE_L/dk) / (2 E_T) equals 1; E_L is the mean of the three
    longitudinal spectra E[a, a], E_T the mean of the six transverse ones
    E[c, a], c != a.  The slope is the central difference in log-log space,
    k dE_L/dk = E_L(k) (ln E_L(k+1) - ln E_L(k-1)) / (ln(k+1) - ln(k-1)), exact
    for power laws.  Defined for 2 <= k <= K-2 with E_L(k +- 1) > 0 and
    E_T(k) > 0, NaN elsewhere.
    """
    E = np.asarray(E, dtype=np.float64)
    EL = (E[0, 0] + E[1, 1] + E[2, 2]) / 3.0
    ET = (E[1, 0] + E[2, 0] + E[0, 1] + E[2, 1] + E[0, 2] + E[1, 2]) / 6.0
    K = EL.size
    ic = np.full(K, np.nan)
    for k in range(2, K - 1):
        if EL[k + 1] > 0.0 and EL[k - 1] > 0.0 and ET[k] > 0.0:
            slope = (np.log(EL[k + 1]) - np.log(EL[k - 1])) / (np.log(k + 1.0) - np.log(k - 1.0))
            ic[k] = (EL[k] - EL[k] * slope) / (2.0 * ET[k])
    return ic
