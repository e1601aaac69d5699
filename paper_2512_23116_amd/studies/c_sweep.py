"""LES spectral analysis: the Smagorinsky constant against a reference DNS
(Sec. 3.4 "LES spectral analysis", Fig. c_variation).

The paper runs LES on 128^3 at Re = 5000 with C = 0, 0.1, 0.16 and 0.25 and
compares the energy spectra with a reference DNS: C = 0 (no eddy viscosity on
the coarse grid) piles energy up at high wavenumbers, C = 0.25 over-dissipates
the small scales, and C = 0.16 lies between.  Setup as in Sec. 3.1: U0 = 0.043,
tau0 = 1/2 + 3 U0 N / Re, three-mode forcing of eq. forcing_pattern with
F0 = C_f U0^2 / N (C_f = 0.2), Taylor-Green start of amplitude U0, t0 = 1000
iterations on every grid; nu_t = C^2 |S| (the form that reproduces the
paper's theta statistics).  The reference DNS is 512^3 at the same Re (the
paper does not state the resolution of its reference curve; 256^3 is itself
under-resolved at Re = 5000 and carries too much energy at high k), run with
two steps per pass: about 16 minutes on one MI355X, the LES runs 15 s each.

Both grids span the same 2 pi box, so shell k is the same wavenumber on both
and E(k) (shell energy of 1/2 |u_hat|^2 in lattice velocity units, U0 the same
on both grids) compares directly.  Spectra are averaged over t/t0 in
[t_start, t_end]; the study reports E(k) and the ratio LES / DNS.

    python -m paper_2512_23116_amd.studies.c_sweep [--t-end 300]
    python -m paper_2512_23116_amd.studies.c_sweep --N-dns 0 > les.json       # LES only
    python -m paper_2512_23116_amd.studies.c_sweep --N-dns 512 --Cs "" > dns512.json
    python -m paper_2512_23116_amd.studies.c_sweep --combine les.json dns512.json
"""
import argparse
import json
import sys
import time

import numpy as np

RATIO_K = (2, 4, 8, 16, 24, 32, 48, 64)


def spectrum_run(N, Re, C, t_start, t_end, every, log, kind):
    import torch
    from .. import lbm, params
    from ..inputs import paper_modes
    stream = torch.cuda.Stream()
    tb = 2 if kind == "dns" else 0
    lat = lbm.Lattice((N, N, N), params.tau0_from_re(N, Re), C,
                      paper_modes(params.forcing_amplitude(N)), precision="fp32",
                      streaming="ab" if tb else "aa", smag_form=1, steps_per_graph=64,
                      temporal_block=tb, stream=stream)
    lat.init(lbm.LBM_INIT_TGV3D, params.U0)
    t0 = 1000
    tic = time.time()
    chunk = 25 * t0
    while lat.steps < t_start * t0:
        lat.step(min(chunk, t_start * t0 - lat.steps))
        lat.sync()
        log(f"{kind} {N}^3 C {C:g}: t/t0 = {lat.steps / t0:g}, {time.time() - tic:.0f} s")
    kmax = N // 2
    E = np.zeros(kmax + 1)
    n = 0
    stats = []
    for step in range(t_start * t0, t_end * t0 + 1, every):
        if step > lat.steps:
            lat.step(step - lat.steps)
        E += lat.spectrum(kmax)
        stats.append(lat.stats())
        n += 1
        if n % 10 == 0:
            log(f"{kind} {N}^3 C {C:g}: window t/t0 = {step / t0:g}, {time.time() - tic:.0f} s")
    lat.close()
    E /= n
    log(f"{kind} {N}^3 Re {Re:g} C {C:g}: {n} spectra in {time.time() - tic:.0f} s")
    return dict(N=N, Re=Re, C=C, snapshots=n, E=[float(v) for v in E],
                energy=float(np.mean([s["energy"] for s in stats])),
                theta_mean=float(np.mean([s["theta_mean"] for s in stats])),
                wall_s=time.time() - tic)


def ratios(les, dns):
    """E_LES(k) / E_DNS(k) at the RATIO_K shells present on the LES grid."""
    El, Ed = np.array(les["E"]), np.array(dns["E"])
    return {int(k): float(El[k] / Ed[k]) for k in RATIO_K if k < El.size}


def run(N_les=128, N_dns=512, Re=5000.0, Cs=(0.0, 0.1, 0.16, 0.25), t_start=200, t_end=300,
        every=2000, log=lambda m: print(m, file=sys.stderr, flush=True)):
    """Reference DNS (N_dns = 0: none) and the LES runs for each C in Cs."""
    dns = spectrum_run(N_dns, Re, 0.0, t_start, t_end, every, log, "dns") if N_dns else None
    les = []
    for C in Cs:
        r = spectrum_run(N_les, Re, C, t_start, t_end, every, log, "les")
        if dns is not None:
            r["ratio_to_dns"] = ratios(r, dns)
        les.append(r)
    return dict(Re=Re, window=[t_start, t_end], every=every, dns=dns, les=les)


def combine(les_result, dns_result):
    """The LES runs of one study output against the reference DNS of another
    (same Re and window), e.g. a finer DNS run on its own."""
    assert les_result["Re"] == dns_result["Re"] and les_result["window"] == dns_result["window"]
    dns = dns_result["dns"]
    les = [dict(r, ratio_to_dns=ratios(r, dns)) for r in les_result["les"]]
    return dict(les_result, dns=dns, les=les)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N-les", type=int, default=128)
    ap.add_argument("--N-dns", type=int, default=512, help="0: no reference DNS")
    ap.add_argument("--Cs", default="0,0.1,0.16,0.25", help="comma list; empty: no LES")
    ap.add_argument("--Re", type=float, default=5000.0)
    ap.add_argument("--t-start", type=int, default=200)
    ap.add_argument("--t-end", type=int, default=300)
    ap.add_argument("--every", type=int, default=2000)
    ap.add_argument("--combine", nargs=2, metavar=("LES_JSON", "DNS_JSON"),
                    help="no GPU: ratios of the LES runs of one output to the DNS of another")
    a = ap.parse_args()
    if a.combine:
        les, dns = (json.load(open(f)) for f in a.combine)
        print(json.dumps(combine(les, dns)), flush=True)
        return
    import torch
    torch.cuda.set_device(0)
    Cs = tuple(float(c) for c in a.Cs.split(",") if c.strip())
    print(json.dumps(run(a.N_les, a.N_dns, a.Re, Cs, t_start=a.t_start, t_end=a.t_end,
                         every=a.every)), flush=True)


if __name__ == "__main__":
    main()
