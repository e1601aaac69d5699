"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bars: FP64 storage, one step from the same state: max error <= 1e-12 of the
deviation scale.  FP32 storage, 10 steps from the same start: <= 1e-5.
Streaming schemes (AA, A/B), graph replay and checkpoints: bitwise.
"""
import math

import numpy as np
import pytest

from oracle import init_fields as I
from oracle import ref_numpy as R
from oracle import stats as ST
from tests.helpers import forced_modes, gpu_available, rel_err

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    m.lib()
    return m


def _lat(lbm, shape, tau0, C, modes=(), **kw):
    return lbm.Lattice(shape, tau0, C, modes, **kw)


# --------------------------------------------------------- FP64 parity ---

@pytest.mark.parametrize("streaming", ["aa", "ab"])
def test_c1_taylor_green_fp64_one_step(lbm, orc, streaming):
    """32^3 TGV (u0 = 0.02), tau0 = 0.51, C = 0.1, no forcing, 200 steps:
    one-step error at steps 0, 1, 10, 100, 199 and the end-to-end error."""
    shape = (32, 32, 32)
    lat = _lat(lbm, shape, 0.51, 0.1, precision="fp64", streaming=streaming)
    lat.init(lbm.LBM_INIT_TGV3D, 0.02)
    olat = orc.Lattice(shape, 0.51, 0.1)
    f0 = olat.init(I.KIND_TGV3D, 0.02)
    assert rel_err(lat.populations(), f0) < 1e-13
    done = 0
    for n in (0, 1, 10, 100, 199):
        lat.step(n - done)
        done = n
        fn = lat.populations()
        lat.step(1)
        done += 1
        err = rel_err(lat.populations(), olat.step(fn, 1))
        print(f"C1 {streaming} step {n}: one-step error {err:.3e}", flush=True)
        assert err <= 1e-12
    assert lat.steps == 200
    err = rel_err(lat.populations(), olat.step(f0, 200))
    print(f"C1 {streaming}: 200-step end-to-end error {err:.3e}", flush=True)
    assert err <= 1e-10
    lat.close()


@pytest.mark.parametrize("shape,smag,streaming,C", [
    ((20, 17, 28), 0, "aa", 0.13),
    ((20, 17, 28), 1, "ab", 0.13),
    ((9, 33, 65), 0, "ab", 0.13),
    # C = 0: the DNS-MRT limit of the LES (Sec. 2.3), tau_e = tau0 everywhere
    ((20, 17, 28), 0, "aa", 0.0),
    ((9, 33, 65), 1, "ab", 0.0),
])
def test_forced_noise_fp64_one_step(lbm, orc, shape, smag, streaming, C):
    """Ragged non-cubic lattices, 16-mode solenoidal forcing, noise start, LES
    (and its C = 0 DNS limit)."""
    modes = forced_modes(F0=3e-5, seed=7)
    lat = _lat(lbm, shape, 0.505, C, modes, precision="fp64", streaming=streaming,
               smag_form=smag)
    lat.init(lbm.LBM_INIT_NOISE, 0.03, 42)
    olat = orc.Lattice(shape, 0.505, C, modes, smag_form=smag)
    assert rel_err(lat.populations(), olat.init(I.KIND_NOISE, 0.03, 42)) < 1e-13
    for _ in range(4):
        fn = lat.populations()
        lat.step(1)
        err = rel_err(lat.populations(), olat.step(fn, 1))
        assert err <= 1e-12, err
    lat.close()


def test_paper_forcing_fp64_one_step(lbm, orc):
    """The paper's three-mode forcing pattern (eq. forcing_pattern)."""
    from paper_2512_23116_amd.inputs import paper_modes
    shape = (24, 24, 24)
    modes = paper_modes(1e-4)
    lat = _lat(lbm, shape, 0.52, 0.13, modes, precision="fp64")
    lat.init(lbm.LBM_INIT_TGV3D, 0.03)
    olat = orc.Lattice(shape, 0.52, 0.13, modes)
    lat.step(3)
    fn = lat.populations()
    lat.step(1)
    assert rel_err(lat.populations(), olat.step(fn, 1)) <= 1e-12


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (1, 7, 3), (5, 1, 9), (3, 4, 1),
                                   (2, 3, 130)])
def test_degenerate_and_tiny_lattices(lbm, orc, shape):
    modes = [((1, 0, 1), (1e-4, 0, -1e-4), 0.3), ((-2, 1, 0), (0, 5e-5, 5e-5), 1.1)]
    for streaming in ("aa", "ab"):
        lat = _lat(lbm, shape, 0.6, 0.2, modes, precision="fp64", streaming=streaming)
        lat.init(lbm.LBM_INIT_NOISE, 0.05, 3)
        olat = orc.Lattice(shape, 0.6, 0.2, modes)
        f0 = olat.init(I.KIND_NOISE, 0.05, 3)
        lat.step(3)
        assert rel_err(lat.populations(), olat.step(f0, 3)) <= 1e-12
        lat.close()


# --------------------------------------------------------- FP32 parity ---

@pytest.mark.parametrize("streaming", ["aa", "ab"])
@pytest.mark.parametrize("case", ["tgv", "forced", "forced_dns"])
def test_fp32_ten_steps(lbm, orc, streaming, case):
    """FP32 storage over 10 steps; "forced_dns" is the forced case at C = 0."""
    shape = (32, 32, 32) if case == "tgv" else (30, 26, 34)
    modes = () if case == "tgv" else forced_modes(F0=3e-5, seed=11)
    kind, amp = (I.KIND_TGV3D, 0.02) if case == "tgv" else (I.KIND_NOISE, 0.02)
    C = {"tgv": 0.1, "forced": 0.13, "forced_dns": 0.0}[case]
    lat = _lat(lbm, shape, 0.51, C, modes, precision="fp32", streaming=streaming)
    lat.init(kind, amp, 5)
    olat = orc.Lattice(shape, 0.51, C, modes)
    f10 = olat.step(olat.init(kind, amp, 5), 10)
    lat.step(10)
    err = rel_err(lat.populations(), f10)
    rho_o, u_o, _ = olat.fields(f10)
    rho, u = lat.moments()
    uerr = np.sqrt(((u - u_o) ** 2).sum() / (u_o ** 2).sum())
    print(f"FP32 {case} {streaming}: 10-step error {err:.3e}, u L2 error {uerr:.3e}", flush=True)
    assert err <= 1e-5 and uerr <= 1e-5
    lat.close()


# ------------------------------------------- schemes, graphs, checkpoints ---

@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16", "bf16"])
def test_aa_equals_ab_bitwise(lbm, precision):
    shape = (18, 21, 23)
    modes = forced_modes(F0=3e-5, seed=3)
    out = {}
    for streaming in ("aa", "ab"):
        lat = _lat(lbm, shape, 0.507, 0.12, modes, precision=precision, streaming=streaming)
        lat.init(lbm.LBM_INIT_NOISE, 0.03, 9)
        res = []
        for n in (2, 1, 98):
            lat.step(n)
            res.append(lat.populations())
        out[streaming] = res
        lat.close()
    for a, b in zip(out["aa"], out["ab"]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("streaming", ["aa", "ab"])
def test_graph_replay_equals_plain_launches_bitwise(lbm, streaming):
    shape = (16, 20, 24)
    modes = forced_modes(F0=3e-5, seed=5)
    res = []
    for spg in (0, 8, 64):
        lat = _lat(lbm, shape, 0.51, 0.1, modes, precision="fp32", streaming=streaming,
                   steps_per_graph=spg)
        lat.init(lbm.LBM_INIT_NOISE, 0.03, 1)
        lat.step(1)      # start the graphs from odd parity / the second array
        lat.step(150)
        res.append(lat.populations())
        lat.close()
    np.testing.assert_array_equal(res[0], res[1])
    np.testing.assert_array_equal(res[0], res[2])


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("streaming", ["aa", "ab"])
def test_checkpoint_restore_bitwise(lbm, precision, streaming):
    shape = (12, 14, 16)
    modes = forced_modes(F0=3e-5, seed=2)
    a = _lat(lbm, shape, 0.51, 0.1, modes, precision=precision, streaming=streaming)
    a.init(lbm.LBM_INIT_NOISE, 0.03, 4)
    a.step(37)
    buf, steps = a.save()
    a.step(29)
    ref = a.populations()
    b = _lat(lbm, shape, 0.51, 0.1, modes, precision=precision, streaming=streaming)
    b.load(buf, steps)
    b.step(29)
    np.testing.assert_array_equal(b.populations(), ref)
    if precision == "fp16":
        # 16-bit storage survives the canonical FP64 round trip exactly
        c = _lat(lbm, shape, 0.51, 0.1, modes, precision=precision, streaming=streaming)
        c.init(lbm.LBM_INIT_REST, 0.0)
        c.step(37)
        b2 = _lat(lbm, shape, 0.51, 0.1, modes, precision=precision, streaming=streaming)
        b2.load(buf, steps)
        c.set_populations(b2.populations())
        c.step(29)
        np.testing.assert_array_equal(c.populations(), ref)


# ----------------------------------------------------------- diagnostics ---

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-4)])
def test_kt_stats_and_fields_match_oracle(lbm, orc, precision, tol):
    shape = (24, 28, 20)
    modes = forced_modes(F0=3e-5, seed=8)
    lat = _lat(lbm, shape, 0.505, 0.13, modes, precision=precision)
    lat.init(lbm.LBM_INIT_TGV3D, 0.03)
    lat.step(13)
    f = lat.populations()
    olat = orc.Lattice(shape, 0.505, 0.13, modes)
    rho_o, u_o, tau_o = olat.fields(f)
    theta = tau_o - 0.5
    ref = ST.field_stats(theta)
    st = lat.stats()
    assert st["n_cells"] == theta.size and st["steps"] == 13 and st["n_nonfinite"] == 0
    for key in ("mean", "var", "skew", "flat", "min", "max"):
        got = st["theta_" + key]
        assert abs(got - ref[key]) <= tol * abs(ref[key]), (key, got, ref[key])
    s3 = math.sqrt(3.0)
    assert abs(st["kt_mean"] - s3 * ref["mean"]) <= tol * s3 * ref["mean"]
    assert abs(st["kt_var"] - 3 * ref["var"]) <= tol * 3 * ref["var"]
    mtol = 1e-12 if precision == "fp64" else 1e-9
    assert abs(st["mass"] - rho_o.sum()) <= mtol * rho_o.sum()
    mom = (rho_o * u_o).reshape(3, -1).sum(1)
    scale = np.abs(rho_o * u_o).sum()
    np.testing.assert_allclose(st["momentum"], mom, rtol=0, atol=max(tol, 1e-12) * scale)
    e_ref = 0.5 * (u_o * u_o).sum(0).mean()
    assert abs(st["energy"] - e_ref) <= tol * e_ref
    # per-cell fields
    rho, u = lat.moments()
    assert np.abs(rho - rho_o).max() <= tol * 1e-2
    assert np.abs(u - u_o).max() <= tol * np.abs(u_o).max()
    kt = lat.kt_field()
    np.testing.assert_allclose(kt, np.float32(s3 * theta), rtol=max(tol, 2e-7), atol=0)
    # into a caller-owned page-locked buffer: the same values
    import torch
    pinned = torch.empty(kt.size, dtype=torch.float32, pin_memory=True).numpy()
    assert np.array_equal(lat.kt_field(out=pinned), kt)
    # one plane at a time: the same values
    for z in sorted({0, shape[0] // 2, shape[0] - 1}):
        assert np.array_equal(lat.kt_slice(z), kt[z])
    for z in (-1, shape[0]):
        with pytest.raises(lbm.LbmError):
            lat.kt_slice(z)


def test_stats_are_bitwise_reproducible_and_C0_is_dns(lbm):
    shape = (20, 20, 20)
    lat = _lat(lbm, shape, 0.53, 0.0, precision="fp32")
    lat.init(lbm.LBM_INIT_NOISE, 0.02, 6)
    lat.step(5)
    a, b = lat.stats(), lat.stats()
    for key in a:
        if not (isinstance(a[key], float) and math.isnan(a[key])):
            assert a[key] == b[key], key
    assert math.isnan(b["theta_skew"]) and math.isnan(b["kt_flat"])
    assert a["theta_min"] == a["theta_max"] == pytest.approx(0.03, abs=1e-15)
    assert a["theta_var"] == 0 and math.isnan(a["theta_flat"])


def test_nonfinite_state_reports_unstable(lbm):
    shape = (8, 9, 10)
    lat = _lat(lbm, shape, 0.52, 0.1, precision="fp32")
    lat.init(lbm.LBM_INIT_TGV3D, 0.02)
    f = lat.populations()
    f[3, 2, 4, 5] = np.nan
    lat.set_populations(f)
    with pytest.raises(lbm.LbmError) as e:
        lat.stats()
    assert e.value.status == lbm.LBM_ERR_UNSTABLE
    st = lat.stats(allow_unstable=True)
    assert st["n_nonfinite"] == 1


def test_invalid_arguments_are_rejected(lbm):
    with pytest.raises(lbm.LbmError) as e:
        _lat(lbm, (4, 4, 4), 0.5, 0.1)
    assert e.value.status == lbm.LBM_ERR_INVALID_ARG
    with pytest.raises(lbm.LbmError):
        _lat(lbm, (4, 4, 4), 0.6, 0.1, modes=[((3, 0, 0), (1e-5, 0, 0), 0.0)])
    lat = _lat(lbm, (4, 4, 4), 0.6, 0.1)
    with pytest.raises(lbm.LbmError) as e:
        lat.step(1)    # before init
    assert e.value.status == lbm.LBM_ERR_STATE
    lat.init(lbm.LBM_INIT_REST, 0.0)
    with pytest.raises(lbm.LbmError):
        lat.sample([64])
    with pytest.raises(lbm.LbmError):
        lat.step(-1)
