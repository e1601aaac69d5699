"""Iso-Reynolds DNS/LES pair (Sec. 3.1, Sec. 5.2-5.3).

The paper pairs a DNS on 800^3 (tau0 - 1/2 = 5.16e-3) with an LES on 100^3
(tau0 - 1/2 = 6.45e-4, C = 0.13): same U0 = 0.043, grid ratio 8, viscosity
scaled with the grid so Re = U0 N / nu0 = 2e4 for both.  Three-mode forcing of
eq. forcing_pattern with F0 = C_f U0^2 / N, Taylor-Green start of amplitude U0,
t0 = 1000 steps.

Two ways to run it:
- ``--scale 2``: the same two relaxation times on 400^3 (DNS, C = 0) and 50^3
  (LES), grid ratio 8, Re = 1e4, both from the Taylor-Green start;
- ``--refine``: the paper's 800^3 / 100^3 pair at Re = 2e4.  One session cannot
  run the 800^3 DNS from t = 0 to the window (2e5 steps to t/t0 = 200), so it
  starts from a developed flow: a run of the same Re on 400^3 (an LES with
  C = 0.13, or with --coarse-C 0 a DNS) runs for the same physical time (1e5 of its steps, the lattice velocity being the
  same), its velocity and density are interpolated onto 800^3 by their Fourier
  series (spectral_upsample) and the DNS starts from their equilibrium
  (lbm_init_velocity) at t/t0 = t_start, then runs `settle` t0 before the window
  so that its own small scales form.  The LES runs from the Taylor-Green start.

Over the window [t_start, t_end] (units of t0) every `every` steps the device
returns E(k), the turbulence scales (lbm_turbulence) and the structure
functions; the study reports the time-averaged spectrum in Kolmogorov units
(kappa eta, E(kappa) / (eps nu^5)^(1/4), with kappa = 2 pi k / N, E(kappa) the
shell energy divided by the shell width 2 pi / N, nu the molecular
viscosity and eps the injected power <F.u>, which equals the total dissipation
in the steady window), the flatness F4(r)
against r / eta, the ESS exponents, for the DNS the comparison with Pope's model
spectrum (studies/pope.py, Sec. 3.4), and for the LES the statistics of
theta = tau_e - 1/2 (Sec. 5.1).

    python -m paper_2512_23116_amd.studies.iso_re_pair [--scale 2] [--t-end 300]
    python -m paper_2512_23116_amd.studies.iso_re_pair --refine [--t-start 200 --settle 5 --t-end 220]
    python -m paper_2512_23116_amd.studies.iso_re_pair --scale 1 --les-only --t-end 1000
"""
import argparse
import json
import math
import sys
import time

import numpy as np

T0 = 1000
ORDERS = {2: 0, 4: 3, 5: 4, 6: 5}


def spectral_upsample(a, n):
    """The periodic field a (m x m x m, m even) on the n x n x n grid, n a multiple
    of m: its Fourier series with the Nyquist modes (|k| = m/2 on any axis) left
    out, evaluated at the finer points (zero padding).  Band-limited fields below
    the Nyquist wavenumber come out exact to rounding."""
    import scipy.fft as F
    m = a.shape[0]
    assert a.shape == (m, m, m) and m % 2 == 0 and n % m == 0
    h = m // 2
    A = F.rfftn(a, workers=-1)
    src = np.r_[0:h, m - h + 1:m]
    dst = np.r_[0:h, n - h + 1:n]
    B = np.zeros((n, n, n // 2 + 1), dtype=complex)
    B[np.ix_(dst, dst, np.arange(h))] = A[np.ix_(src, src, np.arange(h))]
    del A
    return F.irfftn(B, s=(n, n, n), workers=-1) * (n / m) ** 3


def refined_start(Re=2.0e4, C_coarse=0.13, t_start=200, log=print):
    """Start hook for one_run: the developed flow of an LES at half the
    resolution, run for the physical time of t_start t0, interpolated onto the
    lattice (see the module docstring).  Returns the step count it stands for."""
    def start(lat, log_=log):
        import torch
        from .. import lbm, params
        from ..inputs import paper_modes
        N = lat.shape[0]
        Nc = N // 2
        steps_c = t_start * T0 * Nc // N
        coarse = lbm.Lattice((Nc, Nc, Nc), params.tau0_from_re(Nc, Re), C_coarse,
                             paper_modes(params.forcing_amplitude(Nc)), precision="fp32",
                             streaming="ab", smag_form=1, steps_per_graph=64, temporal_block=2,
                             stream=lat.stream)
        coarse.init(lbm.LBM_INIT_TGV3D, params.U0)
        tic = time.time()
        while coarse.steps < steps_c:
            coarse.step(min(25 * T0, steps_c - coarse.steps))
            coarse.sync()
            log_(f"coarse LES {Nc}^3: {coarse.steps} of {steps_c} steps, {time.time() - tic:.0f} s")
        rho_c, u_c = coarse.moments()
        coarse.close()
        if not (np.isfinite(u_c).all() and np.isfinite(rho_c).all()):
            raise RuntimeError(f"the coarse {Nc}^3 run (C = {C_coarse}) became non-finite")
        del coarse
        torch.cuda.empty_cache()
        u = np.stack([spectral_upsample(u_c[a], N) for a in range(3)])
        rho = spectral_upsample(rho_c, N)
        log_(f"interpolated {Nc}^3 (C = {C_coarse}) -> {N}^3, {time.time() - tic:.0f} s")
        lat.init_velocity(torch.from_numpy(u).cuda(), torch.from_numpy(rho).cuda())
        return t_start * T0
    return start


def one_run(kind, N, tau0, C, t_start, t_end, every, log, start=None, precision="fp32"):
    """A run to t_end, averaged over [t_start, t_end]: from the Taylor-Green start,
    or from start(lattice), which initialises the lattice and returns the step
    count its state stands for (at most t_start t0: the run steps on from there
    to the window)."""
    import torch
    from .. import lbm, params
    from ..inputs import paper_modes
    stream = torch.cuda.Stream()
    tb = 2 if kind == "dns" else 0
    lat = lbm.Lattice((N, N, N), tau0, C, paper_modes(params.forcing_amplitude(N)),
                      precision=precision, streaming="ab" if tb else "aa", smag_form=1,
                      steps_per_graph=64, temporal_block=tb, stream=stream)
    if start is None:
        lat.init(lbm.LBM_INIT_TGV3D, params.U0)
        step0 = 0
    else:
        step0 = start(lat)
    t0 = T0
    tic = time.time()
    chunk = 25 * t0
    while step0 + lat.steps < t_start * t0:
        lat.step(min(chunk, t_start * t0 - step0 - lat.steps))
        lat.sync()
        log(f"{kind} {N}^3: t/t0 = {(step0 + lat.steps) / t0:g}, {time.time() - tic:.0f} s")
    rs = sorted(set(int(r) for r in np.round(np.geomspace(1, N // 2, 14))))
    kmax = N // 2
    E = np.zeros(kmax + 1)
    S = np.zeros((len(rs), 6))
    scales = []
    th = []
    n = 0
    last_log = time.time()
    for step in range(t_start * t0, t_end * t0 + 1, every):
        if step > step0 + lat.steps:
            lat.step(step - step0 - lat.steps)
        E += lat.spectrum(kmax)
        S += lat.structure_functions(rs)
        tb_ = lat.turbulence()
        tb_["t"] = step / t0
        scales.append(tb_)
        log(f"{kind} {N}^3 snapshot t/t0 = {step / t0:g}: resolved dissipation / injection "
            f"{tb_['eps_spec'] / tb_['injection'] if tb_['injection'] else float('nan'):.3f}, "
            f"Re_lambda {tb_['re_lambda']:.1f}")
        if C > 0:
            st = lat.stats()
            th.append((st["theta_mean"], st["theta_var"], st["theta_min"], st["theta_max"]))
        n += 1
        if n % 25 == 0 or time.time() - last_log > 30:
            log(f"{kind} {N}^3: window t/t0 = {step / t0:g}, {time.time() - tic:.0f} s")
            last_log = time.time()
    lat.close()
    E /= n
    S /= n
    nu0 = (tau0 - 0.5) / 3.0
    # the dissipation that sets the Kolmogorov units is the total one, which in the
    # statistically steady window equals the injected power <F.u>; the LES resolves
    # only part of it with nu0 (the rest goes through nu_t), so 2 nu0 sum kappa^2 E
    # would not do for it
    eps = float(np.mean([s["injection"] for s in scales]))
    eta = (nu0 ** 3 / eps) ** 0.25
    k = np.arange(kmax + 1)
    kap = 2 * np.pi * k / N
    out = dict(kind=kind, N=N, tau0=tau0, C=C, Re=0.043 * N / nu0, snapshots=n, precision=precision,
               eps=eps, eps_spec=float(np.mean([s["eps_spec"] for s in scales])),
               eps_strain_plus_sgs=float(np.mean([s["eps_strain"] + s["eps_sgs"] for s in scales])),
               eta=eta, re_lambda=float(np.mean([s["re_lambda"] for s in scales])),
               k_eta=[float(v) for v in kap[1:] * eta],
               # E(kappa) = shell energy / shell width 2 pi / N
               E_kolmogorov=[float(v) for v in E[1:] * N / (2 * np.pi) / (eps * nu0 ** 5) ** 0.25],
               r_over_eta=[float(r / eta) for r in rs],
               F4=[float(v) for v in S[:, 3] / S[:, 0] ** 2], wall_s=time.time() - tic,
               # per snapshot: t/t0, resolved dissipation / injected power, Re_lambda
               series=[[s["t"], s["eps_spec"] / s["injection"] if s["injection"] else None,
                        s["re_lambda"]] for s in scales])
    lo, hi = max(2, int(3 * N / 100)), max(6, int(12 * N / 100))
    sel = [i for i, r in enumerate(rs) if lo <= r <= hi]
    x = np.log(S[sel, 2])
    out["zeta"] = {p: float(np.polyfit(x, np.log(S[sel, c]), 1)[0]) for p, c in ORDERS.items()}
    out["r_fit"] = [lo, hi]
    if C == 0:
        from . import pope
        out["pope"] = pope.compare(out["k_eta"], out["E_kolmogorov"])
    if th:
        a = np.array(th)
        out["theta_mean"] = float(a[:, 0].mean())
        out["theta_var"] = float(a[:, 1].mean())
        out["theta_min"] = float(a[:, 2].min())
        out["theta_max"] = float(a[:, 3].max())
        out["theta_mean_over_theta0"] = out["theta_mean"] / (tau0 - 0.5)
    return out


def run(scale=2, t_start=200, t_end=300, every=1000,
        log=lambda m: print(m, file=sys.stderr, flush=True), refine=False, settle=5,
        coarse_C=0.13, dns_precision="fp32", les_only=False):
    """scale = 800 / N_DNS: 1 is the paper's pair (800^3 / 100^3), 2 is 400^3 / 50^3.
    refine: the paper's pair, the DNS from the interpolated developed flow of a
    coarser LES at t/t0 = t_start and averaged over [t_start + settle, t_end].
    les_only: the LES of the pair alone, from the Taylor-Green start, averaged
    over [t_start, t_end] (its window can then be the paper's whole [200, 1000])."""
    from .. import params
    if refine:
        scale = 1
    N_dns, N_les = 800 // scale, 100 // scale
    Re = 2.0e4 / scale
    tau_dns = params.tau0_from_re(N_dns, Re)       # 0.5 + 5.16e-3 for any scale
    tau_les = params.tau0_from_re(N_les, Re)       # 0.5 + 6.45e-4
    if les_only:
        les = one_run("les", N_les, tau_les, 0.13, t_start, t_end, every, log)
        return dict(scale=scale, Re=Re, window=[t_start, t_end], les=les)
    w0 = t_start + settle if refine else t_start
    les = one_run("les", N_les, tau_les, 0.13, w0, t_end, every, log)
    dns = one_run("dns", N_dns, tau_dns, 0.0, w0, t_end, every, log,
                  start=refined_start(Re, coarse_C, t_start, log) if refine else None,
                  precision=dns_precision)
    t_start = w0
    # the LES spectrum on the DNS's k eta grid (Kolmogorov units, log interpolation)
    kd, Ed = np.array(dns["k_eta"]), np.array(dns["E_kolmogorov"])
    kl, El = np.array(les["k_eta"]), np.array(les["E_kolmogorov"])
    m = (kd >= kl[0]) & (kd <= kl[-1])
    ratio = np.exp(np.interp(np.log(kd[m]), np.log(kl), np.log(El)) - np.log(Ed[m]))
    return dict(scale=scale, Re=Re, window=[t_start, t_end], refined=refine,
                coarse_C=coarse_C if refine else None, les=les, dns=dns,
                les_over_dns_spectrum=dict(k_eta=[float(v) for v in kd[m]],
                                           ratio=[float(v) for v in ratio]))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--scale", type=int, default=2)
    ap.add_argument("--t-start", type=int, default=200)
    ap.add_argument("--t-end", type=int, default=300)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--refine", action="store_true",
                    help="800^3 / 100^3 with the DNS started from an interpolated coarse LES")
    ap.add_argument("--settle", type=int, default=5,
                    help="t0 between the refined start and the window")
    ap.add_argument("--coarse-C", type=float, default=0.13,
                    help="Smagorinsky C of the coarse run of the refined start (0: DNS)")
    ap.add_argument("--dns-precision", default="fp32", choices=("fp32", "fp16", "bf16"),
                    help="storage of the DNS populations (two steps per pass)")
    ap.add_argument("--les-only", action="store_true",
                    help="run the LES of the pair alone over [t-start, t-end]")
    a = ap.parse_args()
    print(json.dumps(run(a.scale, a.t_start, a.t_end, a.every, refine=a.refine,
                         settle=a.settle, coarse_C=a.coarse_C,
                         dns_precision=a.dns_precision, les_only=a.les_only)), flush=True)


if __name__ == "__main__":
    main()
