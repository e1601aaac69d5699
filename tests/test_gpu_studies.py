"""The study modules run end to end on small settings."""
import math

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


def test_precision_study_small():
    from paper_2512_23116_amd.studies import precision
    res = precision.study(32, 40, "fp64", ["fp32", "fp16"], n_snaps=2, log=lambda m: None)
    assert set(res["errors"]) == {"fp32", "fp16"}
    for p, bound in (("fp32", 1e-4), ("fp16", 5e-2)):
        for row in res["errors"][p]:
            assert row["u_l2"] <= bound and row["kt_mean"] <= bound
