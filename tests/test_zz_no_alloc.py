"""The allocation-free theta histogram (lbm_theta_histogram_noalloc, counts in
the library's static device scratch) against lbm_theta_histogram (counts in a
buffer the handle allocates): bitwise equal integer counts on two calls in a
row, the second on a smaller lattice with fewer bins (counters the first call
left in the shared scratch must not leak into it), and the size limit."""
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


def _lattice(lbm, shape, precision, seed):
    lat = lbm.Lattice(shape, 0.505, 0.13, forced_modes(F0=3e-5, seed=seed),
                      precision=precision, smag_form=1)
    lat.init(lbm.LBM_INIT_NOISE, 0.03, seed)
    lat.step(7)
    return lat


def test_noalloc_histogram_matches_the_allocating_one(lbm):
    big = _lattice(lbm, (40, 36, 44), "fp32", 3)
    small = _lattice(lbm, (9, 11, 13), "fp64", 5)
    cases = [(big, 0.0, 4e-3, 400), (small, 2e-3, 9e-3, 37), (big, -1e-3, 2e-2, 4096)]
    for lat, lo, hi, nbins in cases:
        ref = lat.theta_histogram(lo, hi, nbins)
        got = lat.theta_histogram_noalloc(lo, hi, nbins)
        print(f"{lat.shape} nbins {nbins}: counts sum {int(got.sum())}, "
              f"occupied bins {int((got[1:-2] > 0).sum())}", flush=True)
        assert got.shape == ref.shape
        assert np.array_equal(got, ref)
        assert int(got.sum()) == lat.ncell
    # repeated on the same lattice: the scratch is cleared on every call
    assert np.array_equal(small.theta_histogram_noalloc(2e-3, 9e-3, 37),
                          small.theta_histogram(2e-3, 9e-3, 37))
    with pytest.raises(lbm.LbmError) as e:
        small.theta_histogram_noalloc(0.0, 1.0, 4097)
    assert e.value.status == lbm.LBM_ERR_INVALID_ARG
    big.close()
    small.close()
