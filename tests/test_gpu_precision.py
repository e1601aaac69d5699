"""Reduced-precision storage (FP16 / BF16 deviations, FP32 collision): error
against the FP64 oracle is reported and bounded by the storage rounding."""
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
