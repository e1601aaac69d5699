"""Host-side helpers of the studies (no GPU)."""
import numpy as np

from paper_2512_23116_amd.studies.regime import histogram_percentiles


def test_histogram_percentiles_of_a_uniform_sample():
    """Uniform theta on [1, 3) in 20 bins of [0, 4): percentiles interpolate
    linearly inside a bin; under / over bins clamp to the range."""
    rng = np.random.default_rng(1)
    theta = rng.uniform(1.0, 3.0, 200000)
    lo, hi, nb = 0.0, 4.0, 20
    q = np.floor((theta - lo) * nb / (hi - lo)).astype(int)
    counts = np.zeros(nb + 3, dtype=np.int64)
    counts[1:nb + 1] = np.bincount(q, minlength=nb)
    p = histogram_percentiles(counts, lo, hi, (5, 50, 95))
    np.testing.assert_allclose(p, np.percentile(theta, (5, 50, 95)), atol=0.01)
    counts2 = np.zeros(nb + 3, dtype=np.int64)
    counts2[0], counts2[nb + 1] = 10, 10
    assert histogram_percentiles(counts2, lo, hi, (1, 99)) == [lo, hi]


def test_c_sweep_combines_les_and_a_separate_reference():
    from paper_2512_23116_amd.studies.c_sweep import combine
    les = dict(Re=5000.0, window=[200, 300], dns=None,
               les=[dict(C=0.1, E=[0.0] + [2.0] * 64)])
    dns = dict(Re=5000.0, window=[200, 300], dns=dict(N=512, E=[0.0] + [1.0] * 256), les=[])
    out = combine(les, dns)
    assert out["dns"]["N"] == 512
    assert out["les"][0]["ratio_to_dns"] == {k: 2.0 for k in (2, 4, 8, 16, 24, 32, 48, 64)}
