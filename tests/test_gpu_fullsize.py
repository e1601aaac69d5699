"""Full-size checks in the configurations the benchmark times (100^3 and 800^3,
FP32 AA and A/B, FP16 / BF16 AA, 64-step graphs): sampled cells against the
oracle's per-cell collision, and conservation over the whole lattice."""
import numpy as np
import pytest

from oracle import d3q19 as OL
from paper_2512_23116_amd import params
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


def _sample_cells(shape, n, seed):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz // 2), (0, ny - 1, 1)]
    pts += [tuple(int(v) for v in rng.integers(0, (nx, ny, nz))) for _ in range(n)]
    return pts


def _cell(x, y, z, shape):
    nz, ny, nx = shape
    return (x % nx) + nx * ((y % ny) + ny * (z % nz))


def sampled_step_check(lat, olat, shape, pts, precision="fp32"):
    """f_i(x, n+1) from the GPU against the oracle's collision of the cell
    x - c_i at step n, for every sampled x and every i."""
    nbr = []
    for (x, y, z) in pts:
        for a in range(19):
            cx, cy, cz = OL.C[a]
            nbr.append(_cell(x - cx, y - cy, z - cz, shape))
    before = lat.sample(np.array(nbr))
    lat.step(1)
    after = lat.sample(np.array([_cell(x, y, z, shape) for (x, y, z) in pts]))
    worst = 0.0
    scale = np.abs(after - OL.W).max()
    for j, (x, y, z) in enumerate(pts):
        for a in range(19):
            cx, cy, cz = OL.C[a]
            xs, ys, zs = x - cx, y - cy, z - cz
            F = olat.force_at(xs % shape[2], ys % shape[1], zs % shape[0])
            fstar, _, _, _ = olat.collide_cell(before[j * 19 + a], F)
            worst = max(worst, abs(fstar[a] - after[j, a]))
    return worst / scale


# (N, storage, streaming, one-step tolerance, mass tolerance): the benchmark's
# lattices.  The one-step bar is the rounding of the stored result relative to
# the deviation scale: FP32 1e-5; FP16 (11 significant bits) 1e-3; BF16 (8 bits)
# 8e-3.  Mass moves only by the rounding of the stored deviations.
FULLSIZE = [(100, "fp32", "aa", 1e-5, 1e-9), (800, "fp32", "aa", 1e-5, 1e-9),
            (800, "fp32", "ab", 1e-5, 1e-9), (800, "fp16", "aa", 1e-3, 1e-8),
            (800, "bf16", "aa", 8e-3, 1e-6)]


@pytest.mark.parametrize("N,precision,streaming,tol,mass_tol", FULLSIZE)
def test_forced_hit_fullsize(lbm, orc, N, precision, streaming, tol, mass_tol):
    shape = (N, N, N)
    cfg = params.forced_hit(N)
    lat = lbm.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], precision=precision,
                      streaming=streaming, smag_form=cfg["smag_form"], steps_per_graph=64)
    lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
    st0 = lat.stats()
    lat.step(129)          # two graph replays and a plain launch (odd parity next)
    st1 = lat.stats()
    olat = orc.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], smag_form=cfg["smag_form"])
    err = sampled_step_check(lat, olat, shape, _sample_cells(shape, 40, N))
    drift = abs(st1["mass"] - st0["mass"]) / st0["mass"]
    print(f"{N}^3 {precision} {streaming}: sampled one-step error {err:.3e}; mass drift "
          f"{drift:.2e}", flush=True)
    assert err <= tol
    assert drift <= mass_tol
    assert st1["n_nonfinite"] == 0 and st1["theta_min"] >= cfg["tau0"] - 0.5 - 1e-9
    lat.step(1)
    err = sampled_step_check(lat, olat, shape, _sample_cells(shape, 40, N + 1))
    assert err <= tol
    lat.close()


def test_fp64_256_one_step_sampled(lbm, orc):
    """256^3 in FP64 (A/B, 2.5 GB per array): sampled one-step error <= 1e-12."""
    N = 256
    shape = (N, N, N)
    cfg = params.forced_hit(N)
    lat = lbm.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], precision="fp64", streaming="ab",
                      smag_form=cfg["smag_form"])
    lat.init(lbm.LBM_INIT_NOISE, 0.02, cfg["init_seed"])
    lat.step(65)
    olat = orc.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], smag_form=cfg["smag_form"])
    err = sampled_step_check(lat, olat, shape, _sample_cells(shape, 30, 7))
    print(f"256^3 fp64: sampled one-step error {err:.3e}", flush=True)
    assert err <= 1e-12
    lat.close()
