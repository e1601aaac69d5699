"""Energy balance and statistical isotropy of forced HIT (Sec. 2.2 eq. energy_balance,
Sec. 3.2, Sec. 3.3).

The paper checks eps = -dE_k/dt + <F.u> in real space for DNS at Re = 2500 on
128^3 and 256^3 and reports the relative error settling, after t/t0 = 200, near
6-7 % (128^3) and below 3.5 % (256^3).  Setup as in Sec. 3.1: C = 0 (DNS),
tau0 = 1/2 + 3 U0 N / Re with U0 = 0.043, the three-mode forcing of
eq. forcing_pattern with F0 = C_f U0^2 / N (C_f = 0.2), Taylor-Green start of
amplitude U0 (an assumption: the paper gives none), t0 = 1000 steps.

Every `every` steps the device returns E_k = 1/2 <u.u>, <F.u>, the dissipation
from the strain of the non-equilibrium moments eps_strain = 2 nu0 <S:S>, and the
spectral eps = 2 nu0 sum kappa^2 E(k) (lbm_turbulence).  dE_k/dt is the central
difference of E_k over the neighbouring snapshots.  Relative error:
|eps - (<F.u> - dE_k/dt)| / eps, averaged over the window.  Isotropy (Sec. 3.3,
Tab. isotropy_metrics): mean and standard deviation of the directional energy
fractions E_i / E and the mean |b_ij| of the off-diagonal anisotropy over the
window, from the Reynolds stresses lbm_turbulence returns, and during the spin-up
the trajectory of the Lumley invariants (xi, eta) and the largest |E_i/E - 1/3|.  Spectral isotropy
(App. spectral isotropy): the coefficient IC(k) of lbm_spectra_1d, averaged over
the window, with its mean and largest departure from 1 over 2 <= k <= N/4.
Spectrum (Sec. 3.4, Fig. DNS_spectra_validation): the window-averaged shell
spectrum in Kolmogorov units (eps = <F.u>, nu = nu0) against Pope's model
spectrum carrying the same energy and dissipation (studies/pope.py).

    python -m paper_2512_23116_amd.studies.energy_balance [--N 128] [--t-end 400]
"""
import argparse
import json
import sys
import time

import numpy as np


def run(N=128, Re=2500.0, t_start=200, t_end=400, every=1000, amp=None,
        log=lambda m: print(m, file=sys.stderr, flush=True)):
    import torch
    from .. import lbm, params
    from ..inputs import paper_modes
    tau0 = params.tau0_from_re(N, Re)
    F0 = params.forcing_amplitude(N)
    stream = torch.cuda.Stream()
    lat = lbm.Lattice((N, N, N), tau0, 0.0, paper_modes(F0), precision="fp32", streaming="aa",
                      steps_per_graph=64, stream=stream)
    lat.init(lbm.LBM_INIT_TGV3D, params.U0 if amp is None else amp)
    t0 = 1000
    tic = time.time()
    # the spin-up, sampled every `traj_every` t0: the Lumley-triangle trajectory
    # from the Taylor-Green start (Fig. isotropy_validation)
    trajectory = []
    traj_every = max(1, t_start // 40)
    for t in range(0, t_start, traj_every):
        if t * t0 > lat.steps:
            lat.step(t * t0 - lat.steps)
        tb = lat.turbulence()
        trajectory.append(dict(t=float(t), xi=tb["lumley_xi"], eta=tb["lumley_eta"],
                               max_frac_dev=float(np.abs(np.asarray(tb["energy_frac"]) - 1 / 3).max())))
    lat.step(t_start * t0 - every - lat.steps)
    lat.sync()
    log(f"energy balance {N}^3 Re {Re:g}: reached t/t0 = {t_start - every / t0:g} "
        f"in {time.time() - tic:.1f} s")
    rows = []
    spec = np.zeros(N // 2 + 1)
    for step in range(t_start * t0 - every, t_end * t0 + every + 1, every):
        if step > lat.steps:
            lat.step(step - lat.steps)
        tb = lat.turbulence()
        _, ic = lat.spectra_1d(N // 4 + 1)
        spec += lat.spectrum(N // 2)
        rows.append(dict(step=step, E=tb["energy"], P=tb["injection"],
                         eps_strain=tb["eps_strain"], eps_spec=tb["eps_spec"],
                         re_lambda=tb["re_lambda"], eta=tb["eta"],
                         frac=tb["energy_frac"], b=tb["b"], ic=ic))
        if len(rows) % 50 == 0:
            log(f"energy balance {N}^3: t/t0 = {step / t0:g}, {time.time() - tic:.1f} s")
    lat.close()
    spec /= len(rows)
    out = []
    for i in range(1, len(rows) - 1):
        dEdt = (rows[i + 1]["E"] - rows[i - 1]["E"]) / (rows[i + 1]["step"] - rows[i - 1]["step"])
        r = rows[i]
        bal = r["P"] - dEdt
        out.append(dict(t=r["step"] / t0, E=r["E"], P=r["P"], dEdt=dEdt,
                        err_strain=abs(r["eps_strain"] - bal) / r["eps_strain"],
                        err_spec=abs(r["eps_spec"] - bal) / r["eps_spec"],
                        re_lambda=r["re_lambda"], eta=r["eta"], frac=r["frac"], b=r["b"],
                        ic=r["ic"]))
    ic = np.mean([o["ic"] for o in out], axis=0)        # k = 0 .. N/4 + 1
    band = ic[2:N // 4 + 1]
    from . import pope
    nu0 = (tau0 - 0.5) / 3.0
    eps = float(np.mean([r["P"] for r in rows]))
    eta = (nu0 ** 3 / eps) ** 0.25
    k_eta = 2 * np.pi * np.arange(1, N // 2 + 1) / N * eta
    E_kol = spec[1:] * N / (2 * np.pi) / (eps * nu0 ** 5) ** 0.25
    pm = pope.compare(k_eta, E_kol)
    summary = dict(
        N=N, Re=Re, tau0=tau0, F0=F0, window=[t_start, t_end], snapshots=len(out),
        mean_err_eps_strain=float(np.mean([o["err_strain"] for o in out])),
        mean_err_eps_spec=float(np.mean([o["err_spec"] for o in out])),
        mean_re_lambda=float(np.mean([o["re_lambda"] for o in out])),
        mean_eta=float(np.mean([o["eta"] for o in out])),
        energy_frac_mean=[float(v) for v in np.mean([o["frac"] for o in out], axis=0)],
        energy_frac_std=[float(v) for v in np.std([o["frac"] for o in out], axis=0)],
        mean_abs_b_offdiag=[float(v) for v in np.mean([np.abs(o["b"][3:]) for o in out], axis=0)],
        ic_k2_to_kq=[float(v) for v in ic[2:N // 4 + 1]],
        ic_band_mean=float(np.mean(band)), ic_band_max_dev=float(np.max(np.abs(band - 1.0))),
        k_eta=[float(v) for v in k_eta], E_kolmogorov=[float(v) for v in E_kol],
        pope={k: v for k, v in pm.items()},
        lumley_trajectory=trajectory,
        paper_err={128: "6-7 %", 256: "< 3.5 %", 512: "~1 % (Re 5000)"}.get(N),
        wall_s=time.time() - tic)
    return summary, out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--Re", type=float, default=2500.0)
    ap.add_argument("--t-start", type=int, default=200)
    ap.add_argument("--t-end", type=int, default=400)
    ap.add_argument("--every", type=int, default=1000)
    a = ap.parse_args()
    summary, _ = run(a.N, a.Re, a.t_start, a.t_end, a.every)
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
