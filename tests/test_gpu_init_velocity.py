"""lbm_init_velocity: f(x, 0) = f_eq(rho(x), u(x)) (App. A eq. feq) from fields
held on the device, against the oracle's equilibrium of the same fields."""
import numpy as np
import pytest

from oracle import ref_numpy as R
from tests.helpers import gpu_available, rel_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


@pytest.mark.parametrize("precision,streaming,tol", [("fp64", "aa", 1e-14), ("fp64", "ab", 1e-14),
                                                     ("fp32", "aa", 2e-6), ("fp16", "ab", 2e-3)])
@pytest.mark.parametrize("with_rho", [True, False])
def test_init_velocity_is_the_equilibrium_of_the_fields(lbm, precision, streaming, tol, with_rho):
    import torch
    shape = (9, 14, 21)                                  # (nz, ny, nx), ragged
    rng = np.random.default_rng(5)
    u = 0.05 * (2 * rng.random((3,) + shape) - 1)
    rho = 1 + 0.01 * (2 * rng.random(shape) - 1) if with_rho else np.ones(shape)
    lat = lbm.Lattice(shape, 0.6, 0.0, precision=precision, streaming=streaming)
    lat.init(lbm.LBM_INIT_NOISE, 0.03, 3).step(3)        # a state to overwrite
    lat.init_velocity(torch.from_numpy(u).cuda(),
                      torch.from_numpy(rho).cuda() if with_rho else None)
    assert lat.steps == 0
    f_ref = R.feq(rho, u)
    err = rel_err(lat.populations(), f_ref)
    r, v = lat.moments()                                 # no force: u = j / rho
    e_rho = np.abs(r - rho).max()
    e_u = np.abs(v - u).max() / np.abs(u).max()
    print(f"{precision} {streaming} rho={with_rho}: f {err:.2e}, rho {e_rho:.2e}, u {e_u:.2e}",
          flush=True)
    assert err <= tol
    assert e_rho <= 20 * tol and e_u <= 50 * tol
    lat.step(2)                                          # and it steps from there
    assert np.isfinite(lat.populations()).all()
    lat.close()


def test_init_velocity_rejects_host_memory_and_bad_shapes(lbm):
    import torch
    shape = (4, 5, 6)
    lat = lbm.Lattice(shape, 0.6, 0.0, precision="fp64")
    host = np.zeros((3,) + shape)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init_velocity(lat.handle, host.ctypes.data)
    assert e.value.status == lbm.LBM_ERR_INVALID_ARG
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init_velocity(lat.handle, 0)
    assert e.value.status == lbm.LBM_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        lat.init_velocity(torch.zeros((3, 4, 5, 7), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        lat.init_velocity(torch.zeros((3,) + shape, dtype=torch.float32, device="cuda"))
    lat.init_velocity(torch.zeros((3,) + shape, dtype=torch.float64, device="cuda"))
    assert np.allclose(lat.moments()[1], 0.0)
    lat.close()
