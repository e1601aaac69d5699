"""Write the FP64 oracle's reference of the 256^3 reduced-precision study.

Runs the C oracle (only ``oracle/`` and the seeded forcing-table generator are
used) on the forced-HIT LES workload at 256^3: tau0 = 1/2 + 3 U0 N / Re with
U0 = 0.043, Re = 2e4 (Sec. 3.1, Sec. 4), nu_t = (C_s Delta)^2 |S| with
C_s = 0.1, 16-mode solenoidal forcing on |k| <= 2 with F0 = C_f U0^2 / N (eq.
forcing_amplitude, C_f = 0.2), start from rest plus 1e-3 velocity noise, for
1000 steps.  At steps 0, 500 and 1000 it records the domain statistics of
theta = tau_e - 1/2 and K_t (Sec. 5.1), the kinetic energy (eq. energy_balance),
the mass, the shell-binned spectrum E(k) for k <= 64 (eq. integral_length_scale,
squared reading), the velocity at 256 seeded cells and the full populations at
64 of them.  The GPU runs of every storage precision are compared with it
(tests/test_gpu_precision.py).

Usage: python tests/golden/make_precision256_reference.py [--steps 1000] [--every 500]
Output: tests/golden/precision256_oracle.json (rewritten after every snapshot).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import init_fields as I  # noqa: E402
from oracle import physics as P  # noqa: E402
from oracle import ref_c  # noqa: E402
from oracle import stats as ST  # noqa: E402
from paper_2512_23116_amd.inputs import random_solenoidal_modes  # noqa: E402

N = 256
C_SMAG = 0.1
SMAG_FORM = 1          # nu_t = (C_s Delta)^2 |S|
NOISE, INIT_SEED, FORCE_SEED = 1e-3, 42, 1234
KMAX = 64
N_U_SAMPLE, N_F_SAMPLE = 256, 64


def sample_cells():
    """Fixed, seeded cell indices (z, y, x): velocity at all, populations at the first 64."""
    rng = np.random.Generator(np.random.PCG64(11))
    return [[int(v) for v in rng.integers(0, N, 3)] for _ in range(N_U_SAMPLE)]


def snapshot(lat, f, step, cells):
    rho, u, tau = lat.fields(f)
    theta = tau - 0.5
    st = ST.field_stats(theta)
    E = ST.energy_spectrum(u)
    return dict(step=step, theta=st,
                kt=dict(mean=float(np.sqrt(3) * st["mean"]), var=float(3 * st["var"]),
                        flat=st["flat"]),
                energy=float(0.5 * (u * u).sum(0).mean()),
                mass=float(rho.sum()),
                spectrum=[float(v) for v in E[:KMAX + 1]],
                u_sample=[[float(u[a, z, y, x]) for a in range(3)] for z, y, x in cells],
                f_sample=[[float(f[i, z, y, x]) for i in range(19)]
                          for z, y, x in cells[:N_F_SAMPLE]])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "precision256_oracle.json"))
    args = ap.parse_args()
    ref_c.build()
    U0, Re = 0.043, 2.0e4
    tau0 = P.tau0_from_re(U0, N, Re)
    F0 = P.forcing_amplitude(U0, N)
    modes = random_solenoidal_modes(F0, FORCE_SEED)
    lat = ref_c.Lattice((N, N, N), tau0, C_SMAG, modes, smag_form=SMAG_FORM)
    f = lat.init(I.KIND_NOISE, NOISE, INIT_SEED)
    cells = sample_cells()
    out = dict(
        _source=("FP64 C oracle, forced-HIT LES 256^3 (the reduced-precision study's workload); "
                 "written by tests/golden/make_precision256_reference.py, which calls only "
                 "oracle/ and the seeded forcing-table generator"),
        N=N, tau0=tau0, C=C_SMAG, smag_form=SMAG_FORM, F0=F0, noise=NOISE, init_seed=INIT_SEED,
        force_seed=FORCE_SEED, every=args.every, steps=args.steps, threads=ref_c.num_threads(),
        sample_cells_zyx=cells, n_f_sample=N_F_SAMPLE, snapshots=[])

    def save():
        with open(args.out + ".tmp", "w") as fh:
            json.dump(out, fh)
        os.replace(args.out + ".tmp", args.out)

    t0 = time.time()
    out["snapshots"].append(snapshot(lat, f, 0, cells))
    for step in range(args.every, args.steps + 1, args.every):
        f = lat.step(f, args.every)
        out["snapshots"].append(snapshot(lat, f, step, cells))
        out["oracle_seconds"] = time.time() - t0
        save()
        print(f"step {step}: {time.time() - t0:.0f} s", flush=True)
    save()


if __name__ == "__main__":
    main()
