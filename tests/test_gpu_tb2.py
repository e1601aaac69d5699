"""Two steps per pass (temporal_block = 2): same results as single A/B steps."""
import numpy as np
import pytest

from oracle import init_fields as I
from tests.helpers import forced_modes, gpu_available, rel_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


def _pair(lbm, shape, precision, spg, modes, seed=3):
    out = []
    for tb in (0, 2):
        lat = lbm.Lattice(shape, 0.507, 0.12, modes, precision=precision, streaming="ab",
                          smag_form=1, steps_per_graph=spg, temporal_block=tb)
        lat.init(lbm.LBM_INIT_NOISE, 0.03, seed)
        out.append(lat)
    return out


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (5, 9, 130), (33, 17, 65), (40, 70, 64),
                                   (64, 64, 64)])
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_two_step_pass_matches_single_steps(lbm, shape, precision):
    modes = forced_modes(F0=3e-5, seed=9)
    ref, tb = _pair(lbm, shape, precision, 8, modes)
    worst = 0.0
    for n in (2, 1, 3, 24, 19):          # odd counts end with a single step
        ref.step(n)
        tb.step(n)
        assert ref.steps == tb.steps
        a, b = tb.populations(), ref.populations()
        worst = max(worst, rel_err(a, b))
    print(f"TB2 {precision} {shape}: max deviation from single steps {worst:.2e}", flush=True)
    assert worst <= (1e-6 if precision == "fp32" else 2e-3)
    ref.close()
    tb.close()


def test_two_step_pass_matches_oracle(lbm, orc):
    shape = (30, 26, 70)
    modes = forced_modes(F0=3e-5, seed=11)
    lat = lbm.Lattice(shape, 0.51, 0.13, modes, precision="fp32", streaming="ab", smag_form=1,
                      temporal_block=2, steps_per_graph=0)
    lat.init(lbm.LBM_INIT_NOISE, 0.02, 5)
    olat = orc.Lattice(shape, 0.51, 0.13, modes, smag_form=1)
    ref = olat.step(olat.init(I.KIND_NOISE, 0.02, 5), 10)
    lat.step(10)
    err = rel_err(lat.populations(), ref)
    print(f"TB2 fp32 vs oracle, 10 steps: {err:.2e}", flush=True)
    assert err <= 1e-5


def test_two_step_pass_large_lattice_conserves_and_agrees(lbm):
    shape = (256, 256, 256)
    from paper_2512_23116_amd import params
    cfg = params.forced_hit(256)
    lats = []
    for tb in (0, 2):
        lat = lbm.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], precision="fp32",
                          streaming="ab", smag_form=cfg["smag_form"], temporal_block=tb)
        lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
        lat.step(130)
        lats.append(lat)
    rng = np.random.default_rng(0)
    cells = rng.integers(0, 256 ** 3, 4000)
    a, b = lats[1].sample(cells), lats[0].sample(cells)
    err = np.abs(a - b).max() / np.abs(b - np.array([1 / 18] * 6 + [1 / 36] * 12 + [1 / 3])).max()
    s0, s1 = lats[0].stats(), lats[1].stats()
    print(f"TB2 256^3 after 130 steps: sampled deviation {err:.2e}", flush=True)
    assert err <= 1e-6
    assert abs(s1["mass"] - s0["mass"]) <= 1e-9 * s0["mass"]
    for lat in lats:
        lat.close()


def test_two_step_pass_config_checks(lbm):
    with pytest.raises(lbm.LbmError):
        lbm.Lattice((8, 8, 8), 0.51, 0.1, streaming="aa", temporal_block=2)
    with pytest.raises(lbm.LbmError):
        lbm.Lattice((8, 8, 8), 0.51, 0.1, precision="fp64", streaming="ab", temporal_block=2)
    with pytest.raises(lbm.LbmError):
        lbm.Lattice((8, 8, 8), 0.51, 0.1, streaming="ab", temporal_block=2, steps_per_graph=6)
