"""Full-size checks in the configurations the benchmark times (100^3 FP32 A/B and
AA in 500-step graphs; 800^3 FP32 AA and A/B, FP16 / BF16 AA in 64-step graphs):
sampled cells against the oracle's per-cell collision, and conservation over the
whole lattice."""
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
FULLSIZE = [(100, "fp32", "ab", 1e-5, 1e-9), (100, "fp32", "aa", 1e-5, 1e-9),
            (800, "fp32", "aa", 1e-5, 1e-9),
            (800, "fp32", "ab", 1e-5, 1e-9), (800, "fp16", "aa", 1e-3, 1e-8),
            (800, "bf16", "aa", 8e-3, 1e-6)]


@pytest.mark.parametrize("N,precision,streaming,tol,mass_tol", FULLSIZE)
def test_forced_hit_fullsize(lbm, orc, N, precision, streaming, tol, mass_tol):
    shape = (N, N, N)
    cfg = params.forced_hit(N)
    spg = 500 if N == 100 else 64      # the benchmark's graph lengths
    lat = lbm.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], precision=precision,
                      streaming=streaming, smag_form=cfg["smag_form"], steps_per_graph=spg)
    lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
    st0 = lat.stats()
    lat.step(2 * spg + 1)  # two graph replays and a plain launch (odd parity next)
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


def sampled_two_step_check(lat, olat, shape, pts):
    """f_i(x, n+2) from one two-step pass against the oracle: every cell
    y - c_j upstream of y = x - c_i collided at step n, streamed to y, y collided
    at step n+1 and streamed to x."""
    need = sorted({_cell(x - OL.C[i][0] - OL.C[j][0], y - OL.C[i][1] - OL.C[j][1],
                         z - OL.C[i][2] - OL.C[j][2], shape)
                   for (x, y, z) in pts for i in range(19) for j in range(19)})
    before = dict(zip(need, lat.sample(np.array(need))))
    lat.step(2)                      # one pass of the two-step kernel
    after = lat.sample(np.array([_cell(x, y, z, shape) for (x, y, z) in pts]))
    nz, ny, nx = shape
    first = {}

    def collided(cx, cy, cz):        # post-collision f at step n of a cell
        c = _cell(cx, cy, cz, shape)
        if c not in first:
            F = olat.force_at(cx % nx, cy % ny, cz % nz)
            first[c] = olat.collide_cell(before[c], F)[0]
        return first[c]

    worst = 0.0
    scale = np.abs(after - OL.W).max()
    for k, (x, y, z) in enumerate(pts):
        for i in range(19):
            yx, yy, yz = x - OL.C[i][0], y - OL.C[i][1], z - OL.C[i][2]
            g = np.array([collided(yx - OL.C[j][0], yy - OL.C[j][1], yz - OL.C[j][2])[j]
                          for j in range(19)])      # f(y, n+1), pre-collision
            F = olat.force_at(yx % nx, yy % ny, yz % nz)
            pred = olat.collide_cell(g, F)[0][i]
            worst = max(worst, abs(pred - after[k, i]))
    return worst / scale


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 2e-3)])
def test_two_step_pass_fullsize_against_the_oracle(lbm, orc, precision, tol):
    """800^3 A/B with two steps per pass, 64-step graphs (the benchmark's
    configuration): sampled cells after one more pass against two oracle steps.
    FP16 rounds the intermediate level through its codec, hence the wider bar."""
    N = 800
    shape = (N, N, N)
    cfg = params.forced_hit(N)
    lat = lbm.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], precision=precision,
                      streaming="ab", smag_form=cfg["smag_form"], steps_per_graph=64,
                      temporal_block=2)
    lat.init(lbm.LBM_INIT_NOISE, cfg["noise"], cfg["init_seed"])
    st0 = lat.stats()
    lat.step(130)                    # two graph replays and a pass
    st1 = lat.stats()
    olat = orc.Lattice(shape, cfg["tau0"], cfg["C"], cfg["modes"], smag_form=cfg["smag_form"])
    err = sampled_two_step_check(lat, olat, shape, _sample_cells(shape, 24, 3))
    drift = abs(st1["mass"] - st0["mass"]) / st0["mass"]
    print(f"800^3 {precision} two-step pass: sampled error {err:.3e}, mass drift {drift:.2e}",
          flush=True)
    assert err <= tol
    assert drift <= (1e-9 if precision == "fp32" else 1e-8)
    assert st1["n_nonfinite"] == 0
    lat.close()
