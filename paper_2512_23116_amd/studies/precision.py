"""Reduced-precision storage study: FP16 / BF16 deviations against FP64 / FP32.

Populations are stored as RNE(sigma * (f - w rho0)) in FP16 (sigma = 2^15) or
BF16 (sigma = 1); collisions run in FP32 and the domain reductions in FP64.
The same forced-HIT LES (the benchmark workload at this N) runs in every
storage precision from the same seeded start, and at each snapshot the study
compares with the reference precision:
  * spectrum error   max over 1 <= k <= K of |E_p(k) / E_ref(k) - 1| for the
                     bands K = 8, 32 and N/4 (shell-binned E(k) of
                     1/2 |u_hat|^2, host FFT).  Storage rounding adds a
                     white-noise floor, so the error grows where E(k) is small;
  * K_t statistics   relative error of the domain mean, variance and flatness;
  * velocity error   ||u_p - u_ref||_2 / ||u_ref||_2;
  * MLUPS of each precision.

    python -m paper_2512_23116_amd.studies.precision --N 256 --steps 5000 --ref fp64
    python -m paper_2512_23116_amd.studies.precision --N 800 --steps 2000 --ref fp32
"""
import argparse
import json
import sys
import time

import numpy as np


def spectrum(u, workers=16):
    """E(k) = 1/2 sum |u_hat|^2 over shells k - 1/2 <= |k| < k + 1/2, u_hat = N^-3 FFT(u)."""
    import scipy.fft as sf
    _, nz, ny, nx = u.shape
    n = nx * ny * nz
    kz = np.fft.fftfreq(nz, 1.0 / nz).astype(np.float32)
    ky = np.fft.fftfreq(ny, 1.0 / ny).astype(np.float32)
    kx = np.arange(nx // 2 + 1, dtype=np.float32)
    shell = np.floor(np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2
                             + kx[None, None, :] ** 2) + 0.5).astype(np.int64)
    # rfft keeps kx >= 0: modes 0 < kx < nx/2 stand for a conjugate pair
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    E = np.zeros(int(shell.max()) + 1)
    for a in range(3):
        uh = sf.rfftn(u[a], workers=workers) / n
        e = 0.5 * (uh.real ** 2 + uh.imag ** 2) * w[None, None, :]
        E += np.bincount(shell.ravel(), weights=e.ravel(), minlength=E.size)
        del uh, e
    return E


def run_precision(N, precision, steps, snaps, log):
    import torch
    from .. import lbm, params
    cfg = params.forced_hit(N)
    stream = torch.cuda.Stream()
    lat = lbm.Lattice((N, N, N), cfg["tau0"], cfg["C"], cfg["modes"], precision=precision,
                      streaming="aa", smag_form=cfg["smag_form"], steps_per_graph=64,
                      stream=stream)
    lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
    out = {}
    kern = 0.0
    for s in snaps:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lat.step(s - lat.steps)
        e1.record(stream)
        e1.synchronize()
        kern += e0.elapsed_time(e1) / 1e3
        st = lat.stats()
        _, u = lat.moments()
        out[s] = dict(stats=st, u=u.astype(np.float32))
        log(f"  {precision} {N}^3 step {s}: <K_t> = {st['kt_mean']:.6e}")
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out, N ** 3 * snaps[-1] / kern / 1e6


def rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else float("nan")


def study(N, steps, ref, precisions, n_snaps=3, log=lambda m: print(m, file=sys.stderr, flush=True)):
    snaps = sorted({int(round(steps * (i + 1) / n_snaps)) for i in range(n_snaps)})
    runs, mlups, spectra = {}, {}, {}
    for p in [ref] + [p for p in precisions if p != ref]:
        runs[p], mlups[p] = run_precision(N, p, steps, snaps, log)
        spectra[p] = {s: spectrum(runs[p][s]["u"]) for s in snaps}
    kmax = N // 4
    res = dict(N=N, steps=steps, reference=ref, snapshots=snaps, mlups=mlups, errors={})
    for p in precisions:
        if p == ref:
            continue
        rows = []
        for s in snaps:
            Er, Ep = spectra[ref][s][1:kmax + 1], spectra[p][s][1:kmax + 1]
            sr, sp = runs[ref][s]["stats"], runs[p][s]["stats"]
            ur, up = runs[ref][s]["u"].astype(np.float64), runs[p][s]["u"].astype(np.float64)
            bands = {f"spectrum_k{K}": float(np.max(np.abs(Ep[:K] / Er[:K] - 1.0)))
                     for K in sorted({8, 32, kmax}) if K <= kmax}
            rows.append(dict(step=s, **bands,
                             kt_mean=rel(sp["kt_mean"], sr["kt_mean"]),
                             kt_var=rel(sp["kt_var"], sr["kt_var"]),
                             kt_flat=rel(sp["kt_flat"], sr["kt_flat"]),
                             energy=rel(sp["energy"], sr["energy"]),
                             u_l2=float(np.sqrt(((up - ur) ** 2).sum() / (ur ** 2).sum()))))
        res["errors"][p] = rows
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--ref", default="fp64")
    ap.add_argument("--precisions", default="fp32,fp16,bf16")
    ap.add_argument("--snaps", type=int, default=3)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    t = time.time()
    res = study(a.N, a.steps, a.ref, a.precisions.split(","), a.snaps)
    res["wall_s"] = time.time() - t
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
