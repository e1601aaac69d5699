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


def _pair(lbm, shape, precision, spg, modes, seed=3, C=0.12, smag_form=1, tau_mode=0):
    out = []
    for tb in (0, 2):
        lat = lbm.Lattice(shape, 0.507, C, modes, precision=precision, streaming="ab",
                          smag_form=smag_form, steps_per_graph=spg, temporal_block=tb,
                          tau_mode=tau_mode)
        lat.init(lbm.LBM_INIT_NOISE, 0.03, seed)
        out.append(lat)
    return out


# Bars: FP32 rounding of the collision, which the compiler may contract
# differently in the two kernels; for 16-bit storage one rounding flip of a
# stored value (FP16 10 significand bits, BF16 7: eight times wider).
BAR = {"fp32": 1e-6, "fp16": 2e-3, "bf16": 1.6e-2}


def _compare(lbm, ref, tb, label):
    worst = 0.0
    for n in (2, 1, 3, 24, 19):          # odd counts end with a single step
        ref.step(n)
        tb.step(n)
        assert ref.steps == tb.steps
        a, b = tb.populations(), ref.populations()
        worst = max(worst, rel_err(a, b))
    print(f"TB2 {label}: max deviation from single steps {worst:.2e}", flush=True)
    ref.close()
    tb.close()
    return worst


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (5, 9, 130), (33, 17, 65), (40, 70, 64),
                                   (64, 64, 64)])
@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_two_step_pass_matches_single_steps(lbm, shape, precision):
    modes = forced_modes(F0=3e-5, seed=9)
    ref, tb = _pair(lbm, shape, precision, 8, modes)
    assert _compare(lbm, ref, tb, f"{precision} {shape}") <= BAR[precision]


@pytest.mark.parametrize("C,smag_form,tau_mode", [(0.0, 1, 0), (0.12, 0, 0), (0.12, 1, 1),
                                                  (0.3, 0, 1)])
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_two_step_pass_follows_every_collision_option(lbm, C, smag_form, tau_mode, precision):
    """The DNS limit C = 0 (the iso-Reynolds DNS runs this way), the linear and the
    C_s^2 Smagorinsky forms and both tau_e modes, on a ragged lattice of several
    tiles and z chunks."""
    modes = forced_modes(F0=3e-5, seed=13)
    ref, tb = _pair(lbm, (37, 31, 70), precision, 8, modes, seed=4, C=C, smag_form=smag_form,
                    tau_mode=tau_mode)
    label = f"{precision} C={C} form={smag_form} tau_mode={tau_mode}"
    assert _compare(lbm, ref, tb, label) <= BAR[precision]


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
