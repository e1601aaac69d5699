"""Pope's model spectrum (host-side study helper): pinned on its published
high-Reynolds-number constants and its defining constraints."""
import numpy as np

from paper_2512_23116_amd.studies import pope


def test_high_reynolds_constants_are_popes():
    """K = Re_lambda sqrt(3/20) at Re_lambda = 1e4: c_L -> 6.78, c_eta -> 0.40."""
    c_L, c_eta, L = pope.constants(1e4 * np.sqrt(3 / 20))
    assert abs(c_L - 6.78) < 0.05 and abs(c_eta - 0.40) < 0.005, (c_L, c_eta)


def test_model_carries_energy_and_dissipation_and_has_a_k41_range():
    K = 300.0
    c_L, c_eta, L = pope.constants(K)
    x = np.geomspace(1e-10, 60.0, 200001)
    m = pope.model(x, L, c_L, c_eta)
    assert abs(np.trapezoid(m, x) / K - 1) < 1e-4
    assert abs(2 * np.trapezoid(x * x * m, x) - 1) < 1e-4
    # at high Reynolds number, between the energy-containing and dissipation
    # ranges, E -> C_K x^(-5/3)
    c_L, c_eta, L = pope.constants(1e4 * np.sqrt(3 / 20))
    xi = 3e-3
    assert abs(pope.model(xi, L, c_L, c_eta) / (1.5 * xi ** (-5 / 3)) - 1) < 0.01


def test_compare_recovers_a_model_spectrum():
    """A spectrum sampled from the model itself on a shell grid compares to ~0
    (up to the energy sum on a discrete grid)."""
    K = 60.0
    c_L, c_eta, L = pope.constants(K)
    x1 = 0.002
    x = x1 * np.arange(1, 2000)
    E = pope.model(x, L, c_L, c_eta)
    r = pope.compare(x, E)
    assert abs(r["K"] / K - 1) < 0.01
    assert r["mean_abs_log_ratio"] < 0.01 and r["shells_in_band"] > 100


def test_compare_reports_when_the_constraints_have_no_solution():
    """Almost no energy for the dissipation: no positive c_L solves the constraints."""
    x = 0.5 * np.arange(1, 40)
    r = pope.compare(x, 1e-6 * np.exp(-x))
    assert r["converged"] is False and "did not converge" in r["error"]
