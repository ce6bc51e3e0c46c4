"""Shared helpers for the GPU tests: problem setup on both sides and comparisons."""
import numpy as np

from oracle import rime
from paper_1910_13908_amd import synth


def setup(cfg, seed=0, noise=True):
    """Oracle side of a problem: obs, V (complex), C (complex, all clusters)."""
    ob = synth.make_obs(cfg, seed=seed, with_noise=noise)
    V, C = rime.make_vis(ob)
    return ob, V, C


def to_dev(ctx_mod, ob, precision, V=None, noise=None):
    """Device copies of a synth.Obs (and optionally of V or the noise) for the library."""
    import torch
    dd = ctx_mod
    obs = dd.device_obs(ob)
    sky = dd.device_sky(ob)
    dt = torch.float32 if precision == dd.MIXED else torch.float64
    out = {"obs": obs, "sky": sky, "dt": dt}
    if V is not None:
        out["V"] = torch.as_tensor(dd.planes(V), dtype=dt, device="cuda").contiguous()
    if noise is not None:
        out["noise"] = torch.as_tensor(dd.planes(noise), dtype=dt, device="cuda").contiguous()
    out["J_true"] = torch.as_tensor(dd.jones_real(ob.jones_true), dtype=torch.float64,
                                    device="cuda").contiguous()
    return out


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
