"""Structure functions, flatness and extended self-similarity (Sec. 5.3).

The paper computes longitudinal structure functions S_p(r) and the flatness
F_4(r) = S_4 / S_2^2 (eq. flatness): F_4 is well above the Gaussian 3 at small r
and relaxes towards 3 at large r, and the ESS exponents zeta_p of
S_p ~ |S_3|^zeta_p follow the She-Leveque model zeta_p = p/9 + 2 (1 - (2/3)^(p/3))
for DNS, closer to K41 (p/3) for p >= 4 in LES.

Two setups (t0 = 1000 steps, Taylor-Green start of amplitude U0 = 0.043, the
three-mode forcing of eq. forcing_pattern):
  les: 100^3, Re = 2e4 (tau0 - 1/2 = 6.45e-4), C = 0.13 in nu_t = (C Delta)^2 |S|
  dns: 256^3, Re = 2500, C = 0
S_p(r) are averaged over snapshots every `every` steps in [t_start, t_end] (units
of t0); zeta_p is the least-squares slope of log S_p against log |S_3| over the
separations in [r_lo, r_hi].

    python -m paper_2512_23116_amd.studies.intermittency --case les|dns
"""
import argparse
import json
import sys
import time

import numpy as np

CASES = {
    "les": dict(N=100, Re=2.0e4, C=0.13, smag_form=1, t_start=200, t_end=300, r_fit=(3, 12)),
    "dns": dict(N=256, Re=2500.0, C=0.0, smag_form=0, t_start=200, t_end=250, r_fit=(4, 24)),
}
ORDERS = {2: 0, 4: 3, 5: 4, 6: 5}     # p -> column of lbm_structure_functions (|S_3| is 2)


def she_leveque(p):
    return p / 9.0 + 2.0 * (1.0 - (2.0 / 3.0) ** (p / 3.0))


def run(case="les", t_start=None, t_end=None, every=1000, N=None,
        log=lambda m: print(m, file=sys.stderr, flush=True)):
    import torch
    from .. import lbm, params
    from ..inputs import paper_modes
    cfg = dict(CASES[case])
    N = N or cfg["N"]
    t_start = cfg["t_start"] if t_start is None else t_start
    t_end = cfg["t_end"] if t_end is None else t_end
    tau0 = params.tau0_from_re(N, cfg["Re"])
    stream = torch.cuda.Stream()
    lat = lbm.Lattice((N, N, N), tau0, cfg["C"], paper_modes(params.forcing_amplitude(N)),
                      precision="fp32", streaming="aa", smag_form=cfg["smag_form"],
                      steps_per_graph=64, stream=stream)
    lat.init(lbm.LBM_INIT_TGV3D, params.U0)
    t0 = 1000
    rs = sorted(set(int(r) for r in np.unique(np.round(np.geomspace(1, N // 2, 16)))))
    tic = time.time()
    lat.step(t_start * t0)
    lat.sync()
    log(f"intermittency {case} {N}^3: reached t/t0 = {t_start} in {time.time() - tic:.1f} s")
    acc = np.zeros((len(rs), 6))
    n = 0
    for step in range(t_start * t0, t_end * t0 + 1, every):
        if step > lat.steps:
            lat.step(step - lat.steps)
        acc += lat.structure_functions(rs)
        n += 1
    lat.close()
    S = acc / n
    F4 = S[:, 3] / S[:, 0] ** 2
    lo, hi = cfg["r_fit"]
    sel = [i for i, r in enumerate(rs) if lo <= r <= hi]
    x = np.log(S[sel, 2])
    zeta = {p: float(np.polyfit(x, np.log(S[sel, c]), 1)[0]) for p, c in ORDERS.items()}
    return dict(case=case, N=N, tau0=tau0, C=cfg["C"], window=[t_start, t_end], snapshots=n,
                r=rs, F4=[float(v) for v in F4], r_fit=[lo, hi],
                zeta=zeta, she_leveque={p: she_leveque(p) for p in ORDERS},
                k41={p: p / 3.0 for p in ORDERS}, wall_s=time.time() - tic)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--case", choices=sorted(CASES), default="les")
    ap.add_argument("--t-start", type=int)
    ap.add_argument("--t-end", type=int)
    ap.add_argument("--every", type=int, default=1000)
    a = ap.parse_args()
    print(json.dumps(run(a.case, a.t_start, a.t_end, a.every)), flush=True)


if __name__ == "__main__":
    main()
