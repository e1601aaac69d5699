"""The asynchronous snapshot (lbm_snapshot_begin / lbm_snapshot_end): the
statistics, the K_t plane and the spectrum of the state at lbm_snapshot_begin,
while later steps already run; equal, bit for bit, to the synchronous calls on
the same state, and the stepping is not disturbed."""
import math

import numpy as np
import pytest

from tests.helpers import forced_modes, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


def _same(a, b):
    for key in a:
        if isinstance(a[key], float) and math.isnan(a[key]):
            assert math.isnan(b[key]), key
        else:
            assert a[key] == b[key], key


@pytest.mark.parametrize("precision,streaming", [("fp32", "aa"), ("fp64", "ab"), ("fp16", "aa")])
def test_snapshot_equals_the_synchronous_calls(lbm, precision, streaming):
    shape = (26, 30, 34)
    modes = forced_modes(F0=3e-5, seed=12)
    mk = lambda: lbm.Lattice(shape, 0.505, 0.13, modes, precision=precision,  # noqa: E731
                             streaming=streaming, smag_form=1, steps_per_graph=16)
    a, b = mk(), mk()
    for lat in (a, b):
        lat.init(lbm.LBM_INIT_NOISE, 0.03, 21)
        lat.step(7)
    kmax, z = 15, 11
    for _ in range(3):
        a.snapshot_begin(kmax, z)
        a.step(16)                      # a graph replay while the snapshot is taken
        st, E, plane = a.snapshot_end()
        ref_st, ref_plane, ref_E = b.stats(), b.kt_slice(z), b.spectrum(kmax)
        _same(st, ref_st)
        assert st["steps"] == b.steps
        assert np.array_equal(plane, ref_plane)
        assert np.array_equal(E, ref_E)
        b.step(16)
    assert a.steps == b.steps
    assert np.array_equal(a.populations(), b.populations())
    # one snapshot at a time; analysis calls wait for its end
    a.snapshot_begin(kmax, z)
    with pytest.raises(lbm.LbmError) as e:
        a.snapshot_begin(kmax, z)
    assert e.value.status == lbm.LBM_ERR_STATE
    with pytest.raises(lbm.LbmError):
        a.spectrum(kmax)
    a.snapshot_end()
    with pytest.raises(lbm.LbmError) as e:
        a.snapshot_end()
    assert e.value.status == lbm.LBM_ERR_STATE
    with pytest.raises(lbm.LbmError):
        a.snapshot_begin(kmax, shape[0])
    for lat in (a, b):
        lat.close()
