"""The spectral interpolation that starts the refined iso-Reynolds DNS
(studies/iso_re_pair.spectral_upsample): exact for band-limited periodic
fields, and it leaves out the Nyquist modes it cannot place."""
import numpy as np

from paper_2512_23116_amd.studies.iso_re_pair import spectral_upsample


def _field(m, n, modes):
    """sum of amp cos(2 pi k.x / m + phase) sampled at x = i m / n, i < n."""
    x = np.arange(n) * (m / n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    out = np.zeros((n, n, n))
    for (kx, ky, kz), amp, ph in modes:
        out += amp * np.cos(2 * np.pi * (kx * X + ky * Y + kz * Z) / m + ph)
    return out


def test_band_limited_field_is_reproduced_on_the_finer_grid():
    m = 12
    modes = [((1, 2, -3), 0.7, 0.3), ((5, 0, 1), -0.2, 1.1), ((0, -5, 4), 0.05, -0.4),
             ((2, 2, 2), 0.3, 0.0), ((0, 0, 0), 1.5, 0.0)]
    for n in (12, 24, 36):
        up = spectral_upsample(_field(m, m, modes), n)
        assert up.shape == (n, n, n)
        assert np.abs(up - _field(m, n, modes)).max() < 1e-12


def test_nyquist_modes_are_left_out():
    m = 8
    band = [((1, -2, 3), 0.4, 0.2), ((0, 1, 0), 1.0, 0.5)]
    nyquist = [((4, 0, 0), 0.3, 0.0), ((1, 4, 2), 0.2, 0.0), ((0, 0, 4), -0.1, 0.0)]
    up = spectral_upsample(_field(m, m, band + nyquist), 16)
    assert np.abs(up - _field(m, 16, band)).max() < 1e-12
