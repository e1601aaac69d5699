"""Batched stepping (continuous batching): each lattice's result is bitwise the
same alone and in any mix, and matches the single-lattice step."""
import numpy as np
import pytest

from tests.helpers import forced_modes, gpu_available, rel_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASES = [((20, 24, 28), 0.51, 0.10, 1), ((32, 32, 32), 0.52, 0.15, 2),
         ((17, 19, 23), 0.505, 0.08, 3), ((8, 8, 8), 0.55, 0.18, 4)]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


def _make(lbm, case, stream):
    shape, tau0, C, seed = case
    lat = lbm.Lattice(shape, tau0, C, forced_modes(F0=3e-5, seed=seed), precision="fp32",
                      stream=stream)
    lat.init(lbm.LBM_INIT_NOISE, 0.03, seed)
    return lat


# per call: the steps each lattice takes (lattices join and leave the mix)
SCHEDULE = [[16, 16, 0, 16], [16, 10, 16, 16], [3, 16, 16, 0], [16, 16, 7, 16], [0, 16, 16, 5]]


def test_batch_isolation_bitwise(lbm):
    import torch
    stream = torch.cuda.Stream()
    mix = [_make(lbm, c, stream) for c in CASES]
    b = lbm.lbm_batch_create(8, 16, stream.cuda_stream)
    for row in SCHEDULE:
        act = [i for i, s in enumerate(row) if s > 0]
        lbm.lbm_batch_step(b, [mix[i].handle for i in act], [row[i] for i in act])
    res_mix = [m.populations() for m in mix]
    steps_mix = [m.steps for m in mix]
    lbm.lbm_batch_destroy(b)
    for i, case in enumerate(CASES):
        alone = _make(lbm, case, stream)
        b1 = lbm.lbm_batch_create(1, 16, stream.cuda_stream)
        for row in SCHEDULE:
            if row[i] > 0:
                lbm.lbm_batch_step(b1, [alone.handle], [row[i]])
        np.testing.assert_array_equal(alone.populations(), res_mix[i])
        assert alone.steps == steps_mix[i]
        lbm.lbm_batch_destroy(b1)
        # the plain single-lattice step gives the same populations
        plain = _make(lbm, case, stream)
        plain.step(steps_mix[i])
        err = rel_err(plain.populations(), res_mix[i])
        print(f"batch case {i}: plain vs batch error {err:.3e}", flush=True)
        assert err <= 1e-6
        alone.close()
        plain.close()
    for m in mix:
        m.close()


def test_batch_rejects_bad_arguments(lbm):
    import torch
    stream = torch.cuda.Stream()
    a = _make(lbm, CASES[0], stream)
    b = lbm.lbm_batch_create(2, 16, stream.cuda_stream)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_batch_step(b, [a.handle], [17])          # more than a graph
    with pytest.raises(lbm.LbmError):
        lbm.lbm_batch_step(b, [a.handle, a.handle], [1, 1])
    other = lbm.Lattice((8, 8, 8), 0.51, 0.1, precision="fp64", stream=stream)
    other.init(lbm.LBM_INIT_REST, 0.0)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_batch_step(b, [other.handle], [2])
    lbm.lbm_batch_destroy(b)
