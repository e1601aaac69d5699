"""Free streaming (lbm_stream_only): the step's data movement with the identity
collision.  After n steps every population has moved n cells along its velocity,
periodically: f_i(x, n) = f_i(x - n c_i, 0), bit for bit in every storage format
and both streaming schemes (the codec round trip of a stored value is exact)."""
import numpy as np
import pytest

from oracle import d3q19 as OL
from tests.helpers import forced_modes, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("streaming", ["aa", "ab"])
def test_free_streaming_is_a_periodic_shift(lbm, precision, streaming):
    shape = (13, 17, 19)
    lat = lbm.Lattice(shape, 0.52, 0.13, forced_modes(F0=3e-5, seed=4), precision=precision,
                      streaming=streaming, smag_form=1)
    lat.init(lbm.LBM_INIT_NOISE, 0.04, 8)
    lat.step(3)                       # a collided state, odd AA parity
    f0 = lat.populations()
    done = 0
    for n in (1, 2, 5):
        lat.stream_only(n - done)
        done = n
        assert lat.steps == 3 + n
        f = lat.populations()
        for i in range(19):
            cx, cy, cz = (int(v) for v in OL.C[i])
            ref = np.roll(f0[i], shift=(n * cz, n * cy, n * cx), axis=(0, 1, 2))
            assert np.array_equal(f[i], ref), (precision, streaming, n, i)
    # and the collision still continues from there
    lat.step(2)
    assert lat.steps == 10 and np.isfinite(lat.populations()).all()
    lat.close()
