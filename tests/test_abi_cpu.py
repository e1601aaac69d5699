"""Host-side checks of the C-ABI library (no GPU work is launched)."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_23116_amd import lbm as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    m.lib()
    return m


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text))


def test_header_declares_what_the_library_exports(lbm):
    declared = header_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T lbm_" in ln}
    assert declared == exported
    assert declared == set(lbm.EXPORTS)
    for name in declared:
        assert hasattr(lbm.lib(), name)


def test_header_compiles_as_c_and_struct_layout_matches(lbm, tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "lbm.h"\n#include <stddef.h>\n#include <stdio.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(lbm_config),'
                   ' sizeof(lbm_force_mode), sizeof(lbm_stats),'
                   ' offsetof(lbm_config, device_buffer_bytes));return 0;}\n')
    exe = tmp_path / "t"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    str(src), "-o", str(exe)], check=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    assert sizes == [ctypes.sizeof(lbm.lbm_config), ctypes.sizeof(lbm.lbm_force_mode),
                     ctypes.sizeof(lbm.lbm_stats), lbm.lbm_config.device_buffer_bytes.offset]


def test_config_defaults_and_required_bytes(lbm):
    c = lbm.lbm_config_default()
    assert (c.nx, c.ny, c.nz) == (32, 32, 32)
    assert c.tau0 == 0.51 and c.smag_C == 0.1 and c.rho0 == 1.0
    assert (c.s_e, c.s_eps, c.s_q, c.s_pi, c.s_m) == (1.19, 1.4, 1.2, 1.4, 1.98)
    assert c.precision == lbm.LBM_FP32 and c.streaming == lbm.LBM_STREAM_AA
    pad = 1728
    plane = 32 ** 3 + pad
    assert lbm.lbm_required_bytes(c) == 19 * plane * 4
    c.streaming = lbm.LBM_STREAM_AB
    c.precision = lbm.LBM_FP64
    assert lbm.lbm_required_bytes(c) == 2 * 19 * plane * 8
    c.nx, c.ny, c.nz = 100, 100, 100
    c.precision, c.streaming = lbm.LBM_FP32, lbm.LBM_STREAM_AA
    assert lbm.lbm_required_bytes(c) == 19 * (1000000 + pad) * 4
    c.nx = c.ny = c.nz = 800
    assert lbm.lbm_required_bytes(c) == 19 * (512000000 + pad) * 4     # 38.9 GB in place
    c.precision = lbm.LBM_BF16_DEV
    assert lbm.lbm_required_bytes(c) == 19 * (512000000 + pad) * 2
    c.nx = 7
    assert lbm.lbm_required_bytes(c) == 19 * ((7 * 800 * 800 + 63) // 64 * 64 + pad) * 2


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("tau0", 0.5), ("tau0", float("nan")), ("smag_C", -0.1), ("precision", 7),
    ("streaming", 2), ("smag_form", 2), ("rho0", 0.0), ("s_m", 2.0), ("storage_scale", 3.0),
    ("steps_per_graph", 3), ("steps_per_graph", 2048), ("n_force_modes", 65),
    ("temporal_block", 3), ("temporal_block", 2), ("tau_mode", 2), ("tau_mode", -1),
])
def test_invalid_configs_are_rejected_on_the_host(lbm, field, value):
    c = lbm.lbm_config_default()
    setattr(c, field, value)
    assert lbm.lbm_required_bytes(c) == 0
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(c)
    assert e.value.status == lbm.LBM_ERR_INVALID_ARG


def test_too_many_cells_and_bad_modes_are_rejected(lbm):
    c = lbm.lbm_config_default()
    c.nx = c.ny = c.nz = 1291          # 1291^3 >= 2^31
    assert lbm.lbm_required_bytes(c) == 0
    c = lbm.lbm_config_default()
    modes = lbm.make_modes([((3, 0, 0), (1e-5, 0, 0), 0.0)])
    c.n_force_modes = 1
    c.force_modes = ctypes.cast(modes, ctypes.POINTER(lbm.lbm_force_mode))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(c)
    assert "k[0]" in str(e.value)


def test_status_strings(lbm):
    L = lbm.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.lbm_status_string(s)
    assert L.lbm_last_error(None) is not None


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    from paper_2512_23116_amd import lbm as m
    monkeypatch.setattr(m, "_lib", None)
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        m.lib()


def test_null_handles_are_rejected_without_touching_a_device(lbm):
    """Every handle-taking entry point returns INVALID_ARG for NULL (no GPU needed)."""
    import numpy as np
    L = lbm.lib()
    d = np.zeros(64)
    dp = d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st = lbm.lbm_stats()
    ts = lbm.lbm_turbulence_stats()
    rs = (ctypes.c_int32 * 1)(1)
    calls = [
        lambda: L.lbm_init_seeded(None, 0, 0.0, 0),
        lambda: L.lbm_step(None, 1),
        lambda: L.lbm_moments(None, dp, dp),
        lambda: L.lbm_kt_stats(None, ctypes.byref(st)),
        lambda: L.lbm_get_populations(None, dp),
        lambda: L.lbm_set_populations(None, dp),
        lambda: L.lbm_spectrum(None, 4, dp),
        lambda: L.lbm_kt_slice(None, 0, np.zeros(4, np.float32).ctypes.data_as(
            ctypes.POINTER(ctypes.c_float))),
        lambda: L.lbm_theta_histogram(None, 0.0, 1.0, 4,
                                      np.zeros(8, np.int64).ctypes.data_as(
                                          ctypes.POINTER(ctypes.c_int64))),
        lambda: L.lbm_spectra_1d(None, 4, dp, dp),
        lambda: L.lbm_structure_functions(None, rs, 1, dp),
        lambda: L.lbm_turbulence(None, 0, ctypes.byref(ts)),
        lambda: L.lbm_synchronize(None),
    ]
    for call in calls:
        assert call() == lbm.LBM_ERR_INVALID_ARG
    assert L.lbm_steps_done(None) == -1 and L.lbm_num_cells(None) == -1
    L.lbm_destroy(None)


def test_kt_field_out_buffer_is_checked_before_the_call(lbm):
    """A caller-supplied K_t buffer of the wrong type, size or layout is refused on
    the host, before the library is entered."""
    import numpy as np
    bad = [np.empty(8, np.float64), np.empty(7, np.float32),
           np.empty((4, 4), np.float32)[:, :2]]
    ro = np.empty(8, np.float32)
    ro.flags.writeable = False
    bad.append(ro)
    for out in bad:
        with pytest.raises(ValueError):
            lbm.lbm_kt_field(None, 8, out)


def test_random_configs_never_crash_and_sizes_follow_the_layout(lbm):
    """Property test over random, mostly invalid configurations: the host-side
    checks either reject them (size 0, INVALID_ARG, no handle) or the state size is
    19 planes of round_up(ncell, 64) + 1728 elements (twice for A/B)."""
    from hypothesis import given, settings, strategies as st
    nan, inf = float("nan"), float("inf")
    floats = st.one_of(st.floats(-3.0, 3.0), st.sampled_from([nan, inf, -inf, 0.5, 0.0, 2.0]))

    @settings(max_examples=300, deadline=None, derandomize=True)
    @given(nx=st.integers(-2, 1400), ny=st.integers(-2, 1400), nz=st.integers(-2, 1400),
           precision=st.integers(-1, 4), streaming=st.integers(-1, 2),
           smag_form=st.integers(-1, 2), tau_mode=st.integers(-1, 2),
           temporal_block=st.integers(-1, 3), spg=st.integers(-2, 2050),
           tau0=floats, C=floats, rho0=floats, s_m=floats, scale=floats)
    def check(nx, ny, nz, precision, streaming, smag_form, tau_mode, temporal_block, spg,
              tau0, C, rho0, s_m, scale):
        c = lbm.lbm_config_default()
        c.nx, c.ny, c.nz = nx, ny, nz
        c.precision, c.streaming, c.smag_form = precision, streaming, smag_form
        c.tau_mode, c.temporal_block, c.steps_per_graph = tau_mode, temporal_block, spg
        c.tau0, c.smag_C, c.rho0, c.s_m, c.storage_scale = tau0, C, rho0, s_m, scale
        size = lbm.lbm_required_bytes(c)
        if size == 0:
            with pytest.raises(lbm.LbmError) as e:
                lbm.lbm_create(c)
            assert e.value.status == lbm.LBM_ERR_INVALID_ARG
            return
        # accepted: every rule of the header holds
        ncell = nx * ny * nz
        assert min(nx, ny, nz) >= 1 and ncell < 2 ** 31
        assert tau0 > 0.5 and C >= 0.0 and rho0 > 0.0 and 0.0 < s_m < 2.0
        assert smag_form in (0, 1) and tau_mode in (0, 1) and streaming in (0, 1)
        assert spg == 0 or (2 <= spg <= 1024 and spg % 2 == 0)
        assert scale == 0.0 or (scale > 0.0 and math.frexp(scale)[0] == 0.5)
        if temporal_block == 2:
            assert streaming == 1 and precision != 0 and spg % 4 == 0
        b = {0: 8, 1: 4, 2: 2, 3: 2}[precision]
        plane = (ncell + 63) // 64 * 64 + 1728
        assert plane * b < 2 ** 32
        assert size == 19 * plane * b * (2 if streaming == 1 else 1)

    check()
