"""The study modules run end to end on small settings."""
import math

import numpy as np
import pytest

from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_regime_study_small():
    from paper_2512_23116_amd.studies import regime
    res = regime.run(smag_form=1, t_start=1, t_end=3, every=1000, N=100, log=lambda m: None)
    w = res["window_mean"]
    assert res["setup"]["snapshots"] == 3
    assert 0 < w["min"] <= w["p5"] <= w["mean"] <= w["p95"] <= w["max"]
    assert math.isfinite(res["normalised_mean"]) and res["normalised_mean"] >= 1.0


def test_regime_reproduces_the_papers_theta_statistics():
    """The paper's LES regime (Sec. 4 setup, Sec. 5.1 result): 100^3, Re 2e4
    (tau0 - 1/2 = 6.45e-4), C = 0.13 in the C_s^2 form, three-mode forcing,
    Taylor-Green start, statistics of theta = tau_e - 1/2 over t/t0 in [200, 600]
    (6e5 steps, 201 snapshots).  The paper prints a domain mean of about 1.34e-3
    (normalised about 2.08), a 95th percentile at or below about 1.82e-3, a 5th
    percentile above 1.0e-3 and no negative values.

    Band: window means move by about 0.5 % between builds whose code generation
    differs (the trajectory is chaotic; 201 snapshots sample it), and the paper
    gives 3 significant figures (+-0.4 %), so the mean and the normalised mean
    must lie within 2 % (4 x the scatter).  The percentiles are read off the
    paper's envelope plot with an approximate sign ("below about 1.82e-3",
    "above 1.0e-3", the latter to 2 figures, +-5 %): p95 <= 1.03 x 1.82e-3,
    p5 >= 0.95 x 1.0e-3.  Every snapshot's minimum must be positive, and the
    largest value stays of the order of the rare peaks the paper reports (global
    maximum about 3.68e-3; one trajectory's extreme is not reproducible, so the
    bound is 1.5 x that)."""
    from paper_2512_23116_amd.studies import regime
    res = regime.run(smag_form=1, C=0.13, t_start=200, t_end=600, every=2000,
                     log=lambda m: print(m, flush=True))
    w = res["window_mean"]
    print({k: w[k] for k in ("mean", "p5", "p50", "p95", "p99", "min", "max")},
          "normalised", res["normalised_mean"], flush=True)
    assert res["setup"]["snapshots"] == 201
    assert abs(w["mean"] / 1.34e-3 - 1.0) <= 0.02
    assert abs(res["normalised_mean"] / 2.08 - 1.0) <= 0.02
    assert w["p95"] <= 1.03 * 1.82e-3
    assert w["p5"] >= 0.95 * 1.0e-3
    assert w["min"] > 0.0 and w["max"] < 1.5 * 3.68e-3
    # the device histogram pools the same cells: its percentiles agree with the
    # snapshot-averaged ones to the bin width (1e-5) and the spread between snapshots
    hp = res["histogram"]["pooled_percentiles"]
    assert abs(hp["p50"] - w["p50"]) <= 2e-5 and abs(hp["p95"] - w["p95"]) <= 3e-5


def test_precision_study_small():
    from paper_2512_23116_amd.studies import precision
    res = precision.study(32, 40, "fp64", ["fp32", "fp16"], n_snaps=2, log=lambda m: None)
    assert set(res["errors"]) == {"fp32", "fp16"}
    for p, bound in (("fp32", 1e-4), ("fp16", 5e-2)):
        for row in res["errors"][p]:
            assert row["u_l2"] <= bound and row["kt_mean"] <= bound


def test_energy_balance_study_small():
    """The balance terms come out finite and positive and the balance closes to
    within 20 % already on 48^3 after a short spin-up (the paper's 128^3 DNS
    settles near 6-7 %)."""
    from paper_2512_23116_amd.studies import energy_balance
    summary, rows = energy_balance.run(N=48, Re=1000.0, t_start=20, t_end=30, every=1000,
                                       log=lambda m: None)
    assert summary["snapshots"] == len(rows) == 11
    for r in rows:
        assert r["E"] > 0 and r["P"] > 0 and math.isfinite(r["dEdt"])
    assert summary["mean_err_eps_strain"] < 0.2, summary
    tr = summary["lumley_trajectory"]
    # the Taylor-Green start has w = 0: E_z = 0, a two-component state
    assert tr[0]["t"] == 0 and abs(tr[0]["max_frac_dev"] - 1 / 3) < 1e-6
    assert tr[-1]["max_frac_dev"] < tr[0]["max_frac_dev"]
    assert len(summary["ic_k2_to_kq"]) == 11
    assert all(math.isfinite(v) and v > 0 for v in summary["ic_k2_to_kq"]), summary
    pm = summary["pope"]
    assert len(summary["E_kolmogorov"]) == 24
    if pm["converged"]:
        assert pm["c_L"] > 0 and pm["c_eta"] > 0 and math.isfinite(pm["mean_abs_log_ratio"])
        assert len(pm["E_model"]) == 24
    print("48^3 short DNS vs Pope's model:", {k: v for k, v in pm.items() if k != "E_model"},
          flush=True)


def test_intermittency_study_small():
    """Short LES run on 48^3: F_4 is finite and above 3 at the smallest separation,
    and the ESS exponents increase with p."""
    from paper_2512_23116_amd.studies import intermittency
    res = intermittency.run("les", t_start=10, t_end=12, every=1000, N=48, log=lambda m: None)
    assert res["snapshots"] == 3
    assert all(math.isfinite(v) for v in res["F4"]) and res["F4"][0] > 3.0
    z = res["zeta"]
    assert z[2] < z[4] < z[5] < z[6]


def test_iso_re_pair_study_small():
    """The DNS/LES pair at 1/16 of the paper's size (50^3 / 6^3), short window:
    both runs report finite Kolmogorov-scaled spectra, F4 and ESS exponents."""
    from paper_2512_23116_amd.studies import iso_re_pair
    res = iso_re_pair.run(scale=16, t_start=2, t_end=3, every=500, log=lambda m: None)
    for kind in ("les", "dns"):
        r = res[kind]
        assert r["snapshots"] == 3 and r["eps"] > 0 and r["eta"] > 0
        assert all(math.isfinite(v) and v > 0 for v in r["E_kolmogorov"])
        assert all(math.isfinite(v) for v in r["F4"])
    assert res["les"]["theta_min"] > 0
    # the LES alone gives the same record (deterministic), and no DNS
    alone = iso_re_pair.run(scale=16, t_start=2, t_end=3, every=500, log=lambda m: None,
                            les_only=True)
    assert "dns" not in alone and alone["window"] == [2, 3]
    assert alone["les"]["E_kolmogorov"] == res["les"]["E_kolmogorov"]
    assert alone["les"]["theta_mean"] == res["les"]["theta_mean"]


def test_c_sweep_study_small():
    """LES C sweep at 32^3 against a 64^3 DNS (Re 1000, short window): finite
    spectra, and at the highest common shell more eddy viscosity leaves less energy."""
    from paper_2512_23116_amd.studies import c_sweep
    res = c_sweep.run(N_les=32, N_dns=64, Re=1000.0, Cs=(0.0, 0.25), t_start=4, t_end=6,
                      every=1000, log=lambda m: None)
    assert res["dns"]["snapshots"] == 3 and len(res["les"]) == 2
    for r in res["les"]:
        assert all(math.isfinite(v) and v >= 0 for v in r["E"])
        assert set(r["ratio_to_dns"]) == {2, 4, 8, 16}
    assert res["les"][1]["E"][16] < res["les"][0]["E"][16]


def test_refined_start_carries_the_coarse_flow_onto_the_fine_lattice():
    """The refined iso-Reynolds start on a small pair: the fine lattice starts
    from the spectral interpolation of the coarse LES's velocity (run here a
    second time, identically), stands for the coarse run's physical time, and
    its step count starts at 0."""
    import torch
    from paper_2512_23116_amd import lbm, params
    from paper_2512_23116_amd.inputs import paper_modes
    from paper_2512_23116_amd.studies import iso_re_pair as P
    N, Re, t_start = 32, 2.0e3, 2
    # unforced, so that its moments give j / rho, the velocity it was started from
    # (with forcing they add the half-force shift F / 2 rho)
    fine = lbm.Lattice((N, N, N), params.tau0_from_re(N, Re), 0.0, precision="fp32",
                       streaming="ab", smag_form=1, temporal_block=2)
    step0 = P.refined_start(Re, 0.13, t_start, log=lambda m: None)(fine)
    assert step0 == t_start * P.T0 and fine.steps == 0
    Nc = N // 2
    coarse = lbm.Lattice((Nc, Nc, Nc), params.tau0_from_re(Nc, Re), 0.13,
                         paper_modes(params.forcing_amplitude(Nc)), precision="fp32",
                         streaming="ab", smag_form=1, temporal_block=2)
    coarse.init(lbm.LBM_INIT_TGV3D, params.U0)
    coarse.step(t_start * P.T0 * Nc // N)
    rho_c, u_c = coarse.moments()
    coarse.close()
    u_ref = np.stack([P.spectral_upsample(u_c[a], N) for a in range(3)])
    rho_f, u_f = fine.moments()
    err = np.abs(u_f - u_ref).max() / np.abs(u_ref).max()
    print(f"refined start: velocity vs the interpolated coarse flow {err:.2e}", flush=True)
    assert err <= 1e-5
    assert np.abs(rho_f - P.spectral_upsample(rho_c, N)).max() <= 1e-6
    # at the coarse points the two differ by the coarse Nyquist modes only
    assert np.abs(u_f[:, ::2, ::2, ::2] - u_c).max() <= 0.1 * np.abs(u_c).max()
    fine.step(4)
    assert np.isfinite(fine.populations()).all()
    fine.close()
    torch.cuda.empty_cache()


def test_one_run_from_a_start_hook_counts_steps_from_the_hooks_time():
    """one_run with the refined start on a small lattice: the state stands for
    t_start t0 steps, so the window's snapshots fall at t_start, t_start + 1/2 and
    t_end without stepping the lattice from 0 again."""
    from paper_2512_23116_amd import params
    from paper_2512_23116_amd.studies import iso_re_pair as P
    N, Re = 32, 2.0e3
    out = P.one_run("dns", N, params.tau0_from_re(N, Re), 0.0, 2, 3, 500, lambda m: None,
                    start=P.refined_start(Re, 0.13, 2, log=lambda m: None))
    assert out["snapshots"] == 3
    assert [s[0] for s in out["series"]] == [2.0, 2.5, 3.0]
    assert all(math.isfinite(s[2]) for s in out["series"])
