"""The plain-C example (paper_2512_23116_amd/examples/forced_hit.c) drives the
C-ABI with no Python or torch in the process (library-owned state, the null
stream, 64-step graph replays); its statistics and spectrum must equal, bit for
bit, those of the same run through the Python binding."""
import os
import subprocess

import pytest

from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "paper_2512_23116_amd", "examples", "forced_hit")


def _parse(out):
    snaps, spec = [], None
    for line in out.splitlines():
        f = line.split()
        if f and f[0] == "step":
            d = {f[i]: float(f[i + 1]) for i in range(2, len(f), 2)}
            d["step"] = int(f[1])
            snaps.append(d)
        elif f and f[0] == "spectrum":
            spec = [float(v) for v in f[1:]]
    return snaps, spec


@pytest.mark.parametrize("precision,scheme", [("fp64", "aa"), ("fp32", "ab")])
def test_c_example_matches_the_python_binding(precision, scheme):
    if not os.path.exists(EXAMPLE):
        pytest.fail("examples/forced_hit is not built (run __graft_entry__.build())")
    # 64 steps per lbm_step call: the example (library-owned state, null stream)
    # replays its 64-step graph on the null stream, the binding on a torch stream
    N, steps, every, C, Re = 24, 192, 64, 0.13, 2.0e4
    r = subprocess.run([EXAMPLE, str(N), str(steps), str(every), precision, scheme, str(C),
                        str(Re)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    snaps, spec = _parse(r.stdout)
    assert [s["step"] for s in snaps] == [0, 64, 128, 192] and spec is not None

    import numpy as np
    from paper_2512_23116_amd import lbm, params
    from paper_2512_23116_amd.inputs import paper_modes
    lbm.lib()
    lat = lbm.Lattice((N, N, N), params.tau0_from_re(N, Re), C,
                      paper_modes(params.forcing_amplitude(N)), precision=precision,
                      streaming=scheme, smag_form=1, steps_per_graph=64)
    lat.init(lbm.LBM_INIT_TGV3D, params.U0)
    for s in snaps:
        lat.step(s["step"] - lat.steps)
        st = lat.stats()
        for key in ("energy", "theta_mean", "theta_var", "kt_mean", "kt_var", "kt_flat", "mass"):
            assert st[key] == s[key] or (np.isnan(st[key]) and np.isnan(s[key])), (key, st[key], s[key])
    # the shell sums run in a fixed order: the spectra are equal bit for bit
    assert list(lat.spectrum(4)[1:]) == spec
    lat.close()
    print(f"C example {precision} {scheme}: <K_t> at step {steps} = {snaps[-1]['kt_mean']:.6e}",
          flush=True)
