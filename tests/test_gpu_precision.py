"""Reduced-precision storage (FP16 / BF16 deviations, FP32 collision): error
against the FP64 oracle is reported and bounded by the storage rounding."""
import os

import numpy as np
import pytest

from oracle import init_fields as I
from tests.helpers import forced_modes, gpu_available, rel_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-5), ("fp16", 5e-3), ("bf16", 5e-2)])
def test_reduced_precision_error_vs_oracle(lbm, orc, precision, bound):
    shape = (32, 32, 32)
    modes = forced_modes(F0=3e-5, seed=21)
    lat = lbm.Lattice(shape, 0.51, 0.13, modes, precision=precision)
    lat.init(lbm.LBM_INIT_TGV3D, 0.03)
    olat = orc.Lattice(shape, 0.51, 0.13, modes)
    f = olat.init(I.KIND_TGV3D, 0.03)
    errs = []
    for n in (1, 10):
        lat.step(n - lat.steps)
        f = olat.step(f, n - (0 if n == 1 else 1))
        errs.append(rel_err(lat.populations(), f))
    rho_o, u_o, tau_o = olat.fields(f)
    rho, u = lat.moments()
    uerr = np.sqrt(((u - u_o) ** 2).sum() / (u_o ** 2).sum())
    st = lat.stats()
    th_err = abs(st["theta_mean"] - (tau_o - 0.5).mean()) / (tau_o - 0.5).mean()
    print(f"{precision}: error after 1 step {errs[0]:.2e}, 10 steps {errs[1]:.2e}, "
          f"u {uerr:.2e}, <theta> {th_err:.2e}", flush=True)
    assert errs[1] <= bound and uerr <= 10 * bound


def test_fp16_scale_keeps_small_deviations(lbm):
    """With sigma = 2^15 deviations of 1e-6 are normal FP16 numbers, not zero."""
    shape = (8, 8, 8)
    lat = lbm.Lattice(shape, 0.6, 0.0, precision="fp16")
    lat.init(lbm.LBM_INIT_SHEAR, 1e-5)
    f = lat.populations()
    g = f - np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3]).reshape(19, 1, 1, 1)
    nz = np.abs(g[0]) > 0
    assert nz.sum() > 0.5 * g[0].size


GOLDEN_256 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "precision256_oracle.json")

# Bars after 1000 steps of the 256^3 workload (laminar spin-up from the noise start,
# where perturbations do not grow), from the rounding each storage format adds per
# step to every stored deviation, accumulated over n = 1000 steps:
#   FP64  any evaluation order, ~1e-16 per step: 1e-10 (populations, velocity),
#         1e-9 (spectrum, theta statistics);
#   FP32  2^-24 relative per step, linear accumulation: n 2^-24 = 6e-5 (populations,
#         velocity), twice that for the quadratic spectrum, 1e-3 for the theta
#         statistics (differences of moments, as in the 10-step K_t parity);
#   FP16  (sigma = 2^15) half an ulp of sigma g is at most 2^-12 of the value,
#         about 4e-4 of the deviation scale per step; a random walk over n steps
#         gives 1.2e-2: bar 3 x that, twice for the spectrum and theta statistics;
#   BF16  half an ulp is 2^-9 of the value, 2e-3 per step, 6e-2 over n steps as a
#         random walk: bar 3 x that.
# The spectrum bar applies to the largest relative error over the shells k <= 64
# for FP64 and FP32.  For the 16-bit formats it applies to the energy-weighted error
# sum_k |E - E_ref| / sum_k E_ref (k <= 64): their rounding acts as white noise on
# the velocity, and shells 3..8 hold ~1e-11 of energy (the forcing feeds k <= 2, the
# noise start fills the high shells), so a per-shell ratio there measures the noise
# floor, which is reported, not bounded.
PRECISION_256_BARS = {
    "fp64": dict(f=1e-10, u=1e-10, spec=1e-9, theta=1e-9),
    "fp32": dict(f=6e-5, u=6e-5, spec=1.2e-4, theta=1e-3),
    "fp16": dict(f=4e-2, u=4e-2, spec=8e-2, theta=8e-2),
    "bf16": dict(f=0.2, u=0.2, spec=0.4, theta=0.4),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "bf16"])
def test_precision_256_against_the_oracle(lbm, precision):
    """The precision-study workload (forced-HIT LES 256^3, 16-mode forcing, 1e-3 noise
    start, C_s = 0.1) in each storage format, 1000 steps, against the FP64 C
    oracle's record of the same run (tests/golden/precision256_oracle.json, written
    by tests/golden/make_precision256_reference.py from oracle/ alone): sampled
    populations and velocities, the spectrum E(k) for k <= 64 and the theta
    statistics at steps 500 and 1000."""
    import json
    from paper_2512_23116_amd.inputs import random_solenoidal_modes
    g = json.load(open(GOLDEN_256))
    if len(g["snapshots"]) < 3:
        pytest.skip("the oracle reference is incomplete")
    N = g["N"]
    modes = random_solenoidal_modes(g["F0"], g["force_seed"])
    lat = lbm.Lattice((N, N, N), g["tau0"], g["C"], modes, precision=precision,
                      streaming="aa", smag_form=g["smag_form"])
    lat.init(lbm.LBM_INIT_NOISE, g["noise"], g["init_seed"])
    zyx = g["sample_cells_zyx"]
    cells = np.array([x + N * (y + N * z) for z, y, x in zyx])
    nf = g["n_f_sample"]
    bars = PRECISION_256_BARS[precision]
    for snap in g["snapshots"][1:]:
        lat.step(snap["step"] - lat.steps)
        st = lat.stats()
        E = lat.spectrum(64)
        f = lat.sample(cells[:nf])
        _, u = lat.moments()
        u_s = np.array([u[:, z, y, x] for z, y, x in zyx])
        f_o = np.array(snap["f_sample"])
        u_o = np.array(snap["u_sample"])
        W = np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3])
        e_f = float(np.abs(f - f_o).max() / np.abs(f_o - W).max())
        e_u = float(np.sqrt(((u_s - u_o) ** 2).sum() / (u_o ** 2).sum()))
        E_o = np.array(snap["spectrum"])
        e_spec = {K: float(np.max(np.abs(E[1:K + 1] / E_o[1:K + 1] - 1))) for K in (8, 32, 64)}
        e_spec_w = float(np.abs(E[1:65] - E_o[1:65]).sum() / E_o[1:65].sum())
        th = snap["theta"]
        e_th = {k: abs(st["theta_" + k] - th[k]) / abs(th[k]) for k in ("mean", "var", "flat")}
        e_E = abs(st["energy"] - snap["energy"]) / snap["energy"]
        print(f"256^3 {precision} step {snap['step']} vs oracle: populations {e_f:.2e}, "
              f"u {e_u:.2e}, spectrum max over k<=8/32/64 {e_spec[8]:.2e}/{e_spec[32]:.2e}/"
              f"{e_spec[64]:.2e}, energy-weighted {e_spec_w:.2e}, theta mean/var/flat "
              f"{e_th['mean']:.2e}/{e_th['var']:.2e}/{e_th['flat']:.2e}, energy {e_E:.2e}",
              flush=True)
        assert e_f <= bars["f"] and e_u <= bars["u"]
        spec_err = e_spec[64] if precision in ("fp64", "fp32") else e_spec_w
        assert spec_err <= bars["spec"] and e_E <= bars["spec"]
        assert max(e_th.values()) <= bars["theta"]
    lat.close()
