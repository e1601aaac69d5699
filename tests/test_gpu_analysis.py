"""On-device spectrum and structure functions against the oracle's definitions
applied to the same velocity field."""
import numpy as np
import pytest

from oracle import stats as ST
from tests.helpers import forced_modes, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


@pytest.mark.parametrize("shape,precision", [((36, 48, 40), "fp64"), ((100, 100, 100), "fp32"),
                                             ((17, 9, 30), "fp64")])
def test_spectrum_and_structure_functions_match_oracle(lbm, shape, precision):
    lat = lbm.Lattice(shape, 0.52, 0.13, forced_modes(F0=3e-5, seed=4), precision=precision,
                      smag_form=1)
    lat.init(lbm.LBM_INIT_TGV3D, 0.03)
    lat.step(40)
    _, u = lat.moments()
    kmax = max(shape) // 2 + 3
    E = lat.spectrum(kmax)
    E_ref = ST.energy_spectrum(u)[:kmax + 1]
    E_ref = np.pad(E_ref, (0, kmax + 1 - E_ref.size))
    np.testing.assert_allclose(E, E_ref, rtol=1e-10, atol=1e-14 * E_ref.max())
    assert abs(E.sum() - 0.5 * (u * u).sum(0).mean()) <= 1e-10 * E.sum() or kmax < max(shape)
    rs = [1, 2, 3, 7, 20, max(shape) + 1]
    S = lat.structure_functions(rs)
    S_ref = ST.structure_functions(u, rs)
    np.testing.assert_allclose(S, S_ref, rtol=1e-9, atol=1e-300)
    F4 = S[:, 3] / S[:, 0] ** 2
    print(f"{shape} {precision}: E(1..4) = {E[1:5]}, F4(r) = {np.round(F4, 3)}", flush=True)
    lat.close()
