"""Shared helpers of the test suite (no method arithmetic here)."""
import numpy as np

from oracle import d3q19 as OL

W4 = OL.W.reshape(19, 1, 1, 1)


def dev_scale(f_ref):
    """Scale of the deviation populations f - w (rho0 = 1)."""
    return float(np.abs(np.asarray(f_ref).reshape((19, -1)) - OL.W.reshape(19, 1)).max())


def rel_err(f, f_ref):
    """max |f - f_ref| / max |f_ref - w|: error relative to the deviation scale."""
    f = np.asarray(f).reshape((19, -1))
    f_ref = np.asarray(f_ref).reshape((19, -1))
    return float(np.abs(f - f_ref).max() / dev_scale(f_ref))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def forced_modes(F0=2e-5, seed=1234):
    from paper_2512_23116_amd.inputs import random_solenoidal_modes
    return random_solenoidal_modes(F0, seed)
