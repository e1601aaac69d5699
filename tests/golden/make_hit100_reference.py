"""Write the FP64 oracle's statistics of the 100^3 forced-HIT LES run.

Runs the C oracle (only ``oracle/`` and the seeded input generator are used)
on the forced-HIT LES workload: 100^3 periodic, tau0 = 1/2 + 3 U0 N / Re with
U0 = 0.043, Re = 2e4 (Sec. 3.1, Sec. 4), nu_t = (C_s Delta)^2 |S| with C_s = 0.1,
16-mode solenoidal forcing on |k| <= 2 with F0 = C_f U0^2 / N (eq.
forcing_amplitude, C_f = 0.2), start from rest plus 1e-3 velocity noise.  Every
500 steps up to 20000 it records the domain statistics of theta = tau_e - 1/2
and K_t (Sec. 5.1), the kinetic energy 1/2 <u.u> (eq. energy_balance), the
shell-binned spectrum E(k) (eq. integral_length_scale, squared reading) and the
velocity at 64 fixed seeded cells (to date where trajectories part).

Turbulence is chaotic, so long runs are compared through statistics only.  A
second run (b) starts from the same state with every population deviation
f_i - w_i rho0 rounded to FP32, a perturbation of the size FP32 storage makes;
the spread between the two runs shows how far two equally valid trajectories
drift apart and sets the comparison band.

Usage: python tests/golden/make_hit100_reference.py [--steps 20000] [--every 500] [--resume]
Output: tests/golden/hit100_oracle_stats.json (rewritten after every snapshot).
``--resume`` keeps runs already complete in the output file (same perturbation,
all snapshots) and computes the others.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import d3q19 as D  # noqa: E402
from oracle import init_fields as I  # noqa: E402
from oracle import physics as P  # noqa: E402
from oracle import ref_c  # noqa: E402
from oracle import stats as ST  # noqa: E402
from paper_2512_23116_amd.inputs import random_solenoidal_modes  # noqa: E402

N = 100
C_SMAG = 0.1
SMAG_FORM = 1          # nu_t = (C_s Delta)^2 |S|
NOISE, INIT_SEED, FORCE_SEED = 1e-3, 42, 1234
KMAX = 25
N_SAMPLE = 64          # cells whose velocity is recorded at every snapshot
PERTURBATION = {
    "a": "none",
    "b": "deviations f_i - w_i rho0 of the initial populations rounded to FP32",
}


def sample_cells():
    """Fixed, seeded cell indices (z, y, x) for the pointwise velocity record."""
    rng = np.random.Generator(np.random.PCG64(7))
    return [[int(v) for v in rng.integers(0, N, 3)] for _ in range(N_SAMPLE)]


def snapshot(lat, f, step, cells):
    rho, u, tau = lat.fields(f)
    theta = tau - 0.5
    st = ST.field_stats(theta)
    E = ST.energy_spectrum(u)
    return dict(step=step, theta=st,
                kt=dict(mean=float(np.sqrt(3) * st["mean"]), var=float(3 * st["var"])),
                energy=float(0.5 * (u * u).sum(0).mean()),
                mass=float(rho.sum()),
                spectrum=[float(v) for v in E[:KMAX + 1]],
                u_sample=[[float(u[a, z, y, x]) for a in range(3)] for z, y, x in cells])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "hit100_oracle_stats.json"))
    ap.add_argument("--resume", action="store_true")
    args = ap.parse_args()
    ref_c.build()
    U0, Re = 0.043, 2.0e4
    tau0 = P.tau0_from_re(U0, N, Re)
    F0 = P.forcing_amplitude(U0, N)
    modes = random_solenoidal_modes(F0, FORCE_SEED)
    lat = ref_c.Lattice((N, N, N), tau0, C_SMAG, modes, smag_form=SMAG_FORM)
    f0 = lat.init(I.KIND_NOISE, NOISE, INIT_SEED)
    w = np.asarray(D.W, dtype=np.float64).reshape(19, 1, 1, 1)
    g0 = w + (f0 - w).astype(np.float32).astype(np.float64)      # rho0 = 1
    out = dict(
        _source=("FP64 C oracle, forced-HIT LES 100^3 (workload of this repository's benchmark); "
                 "written by tests/golden/make_hit100_reference.py, which calls only oracle/ "
                 "and the seeded forcing-table generator"),
        N=N, tau0=tau0, C=C_SMAG, smag_form=SMAG_FORM, F0=F0, noise=NOISE, init_seed=INIT_SEED,
        force_seed=FORCE_SEED, every=args.every, steps=args.steps, threads=ref_c.num_threads(),
        perturbation=dict(PERTURBATION), sample_cells_zyx=sample_cells(), runs={"a": [], "b": []})
    n_snap = args.steps // args.every + 1
    if args.resume and os.path.exists(args.out):
        old = json.load(open(args.out))
        for name in out["runs"]:
            same = old.get("perturbation", {}).get(name, "none" if name == "a" else None)
            if same == PERTURBATION[name] and len(old["runs"].get(name, [])) == n_snap \
                    and old.get("every") == args.every \
                    and old.get("sample_cells_zyx") == out["sample_cells_zyx"]:
                out["runs"][name] = old["runs"][name]
                print(f"run {name}: kept from {args.out}", flush=True)

    def save():
        with open(args.out + ".tmp", "w") as fh:
            json.dump(out, fh)
        os.replace(args.out + ".tmp", args.out)

    for name, f in (("a", f0), ("b", g0)):
        if out["runs"][name]:
            continue
        t0 = time.time()
        out["runs"][name].append(snapshot(lat, f, 0, out["sample_cells_zyx"]))
        for step in range(args.every, args.steps + 1, args.every):
            f = lat.step(f, args.every)
            out["runs"][name].append(snapshot(lat, f, step, out["sample_cells_zyx"]))
            save()
            print(f"run {name} step {step}: {time.time() - t0:.0f} s", flush=True)
    save()


if __name__ == "__main__":
    main()
