"""Whole-lattice parity where the step kernel walks its blocks in 64-block
chunks taken in turn by the 8 XCDs (states above 256 MB), and bitwise
independence of the result from the block order.

Every population of every cell is compared with the oracle (no sampling), on
ragged lattices whose block count leaves both a partial last block and an
incomplete last round of chunks (the blocks that keep the dispatch order).
Bars: FP64 one step <= 1e-12, FP32 ten steps <= 1e-5 of the deviation scale.
"""
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


def _blocks(shape):
    nz, ny, nx = shape
    return (nx * ny * nz + 255) // 256


def test_whole_lattice_fp64_ab_chunked_order(lbm, orc, monkeypatch):
    """130 x 127 x 129 FP64 A/B (2 x 324 MB of state, so the library picks the
    64-block chunked order): 8320 blocks (the last one partly filled) = 16
    complete rounds of 8 x 64 and 128 blocks in dispatch order.  One step by a
    plain launch and one after a 64-step graph replay, each against the oracle's
    step of the GPU's own state."""
    monkeypatch.delenv("LBM_XCD_REMAP", raising=False)
    shape = (130, 127, 129)
    assert _blocks(shape) == 8320 and _blocks(shape) % 512 == 128
    modes = forced_modes(F0=3e-5, seed=17)
    lat = lbm.Lattice(shape, 0.505, 0.13, modes, precision="fp64", streaming="ab",
                      smag_form=1, steps_per_graph=64)
    assert lat.cfg.device_buffer_bytes > 256 << 20
    lat.init(lbm.LBM_INIT_NOISE, 0.03, 23)
    olat = orc.Lattice(shape, 0.505, 0.13, modes, smag_form=1)
    f = lat.populations()
    assert rel_err(f, olat.init(I.KIND_NOISE, 0.03, 23)) < 1e-13
    lat.step(1)
    err0 = rel_err(lat.populations(), olat.step(f, 1))
    lat.step(1)
    lat.step(64)            # one graph replay (the current array is the first again)
    assert lat.steps == 66
    f = lat.populations()
    lat.step(1)
    err1 = rel_err(lat.populations(), olat.step(f, 1))
    print(f"130x127x129 FP64 A/B, chunked order: one-step errors {err0:.3e} (plain launch), "
          f"{err1:.3e} (after a graph replay)", flush=True)
    assert err0 <= 1e-12 and err1 <= 1e-12
    lat.close()


def test_whole_lattice_fp32_aa_chunked_order_ten_steps(lbm, orc, monkeypatch):
    """222 x 224 x 226 FP32 AA (854 MB of state, chunked order): 43901 blocks (the
    last one half full) = 85 complete rounds of 8 x 64 and 381 blocks in dispatch
    order, 10 steps as
    one 10-step graph replay (even and odd AA launches), every population
    against 10 oracle steps from the same start."""
    monkeypatch.delenv("LBM_XCD_REMAP", raising=False)
    shape = (222, 224, 226)
    assert _blocks(shape) == 43901 and _blocks(shape) % 512 == 381
    modes = forced_modes(F0=3e-5, seed=19)
    lat = lbm.Lattice(shape, 0.505, 0.13, modes, precision="fp32", streaming="aa",
                      smag_form=1, steps_per_graph=10)
    assert lat.cfg.device_buffer_bytes > 256 << 20
    lat.init(lbm.LBM_INIT_NOISE, 0.02, 29)
    olat = orc.Lattice(shape, 0.505, 0.13, modes, smag_form=1)
    ref = olat.step(olat.init(I.KIND_NOISE, 0.02, 29), 10)
    lat.step(10)
    f = lat.populations()
    lat.close()
    err = rel_err(f, ref)
    del f
    print(f"222x224x226 FP32 AA, chunked order: 10-step error {err:.3e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("precision,streaming,tb", [("fp32", "aa", 0), ("fp32", "ab", 0),
                                                    ("fp16", "aa", 0), ("fp32", "ab", 2),
                                                    ("fp16", "ab", 2)])
def test_block_order_does_not_change_results(lbm, monkeypatch, precision, streaming, tb):
    """The same lattice stepped with every block order (dispatch order, one range
    per XCD, chunks of 2, 3 and 64 blocks, and the library's default) gives
    bitwise the same populations: 66 x 64 x 67 = 1106 blocks, so the chunked
    orders end in incomplete rounds.  With two steps per pass the orders give
    different launch plans (tile ranges for 8 XCDs, or one range), so the
    results must not depend on the plan either.  Plain launches and graph
    replays both run."""
    shape = (66, 64, 67)
    modes = forced_modes(F0=3e-5, seed=31)
    orders = [None, "0", "1", "2", "3", "64"] if tb == 0 else [None, "0", "1"]
    out = []
    for order in orders:
        if order is None:
            monkeypatch.delenv("LBM_XCD_REMAP", raising=False)
        else:
            monkeypatch.setenv("LBM_XCD_REMAP", order)
        lat = lbm.Lattice(shape, 0.51, 0.13, modes, precision=precision, streaming=streaming,
                          smag_form=1, steps_per_graph=64, temporal_block=tb)
        lat.init(lbm.LBM_INIT_NOISE, 0.03, 37)
        lat.step(4)       # even parity / first array again, also with two steps per pass
        lat.step(64)      # one graph replay
        lat.step(6)
        out.append(lat.populations())
        lat.close()
    monkeypatch.delenv("LBM_XCD_REMAP", raising=False)
    for order, f in zip(orders[1:], out[1:]):
        assert np.array_equal(f, out[0]), f"block order {order} differs from the default"
