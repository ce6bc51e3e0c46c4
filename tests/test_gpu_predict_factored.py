"""Station-factorised predict (ddc_predict_factored) against the FP64 oracle's predict and
against the direct predict, through the C ABI.

The oracle computes each baseline's phase from the baseline coordinates; the factorised
kernel from the two stations' coordinates.  Both give the coherencies of the measurement
equation; the tolerances are those of the direct predict: 1e-11 relative in FP64 (phase
rounding at a few thousand turns), 1e-5 relative for the mixed path (FP32 sin/cos of each
station's phasor and FP32 accumulation).
"""
import numpy as np
import pytest

from oracle import rime
from paper_1910_13908_amd import synth

from _gpu_util import setup, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1910_13908_amd import ddcal
    return ddcal


@pytest.fixture(scope="module")
def ctx(dd):
    c = dd.Context(0)
    yield c
    c.close()


SMALL = synth.ObsConfig(13, 3, 5, 3, (140e6, 160e6), jones_amp=0.2)           # N < one block
POL = synth.ObsConfig(9, 2, 4, 2, (150e6,), polarised=True, jones_amp=0.2)     # four passes
WIDE = synth.ObsConfig(40, 1, 300, 2, (150e6,), disk_radius_m=20000.0)        # many LDS chunks
TWO_BLOCKS = synth.ObsConfig(70, 2, 7, 2, (145e6, 155e6))                      # ragged second block


@pytest.mark.parametrize("cfg", [SMALL, POL, WIDE, TWO_BLOCKS], ids=["small", "polarised", "wide", "two_blocks"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_factored_vs_oracle(dd, ctx, cfg, prec):
    ob, V, C = setup(cfg, seed=5)
    obs, sky = dd.device_obs(ob), dd.device_sky(ob)
    su, sv, sw = dd.device_station_uvw(ob)
    got = dd.unplanes(ctx.predict_factored(obs, su, sv, sw, sky, prec).cpu().numpy())
    tol = 1e-11 if prec == 0 else 1e-5
    for k in range(ob.K):
        assert rel(got[k], C[k]) <= tol, (k, rel(got[k], C[k]))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_factored_empty_cluster(dd, ctx, prec):
    """A cluster without sources has zero coherencies; its neighbours are unaffected."""
    import torch
    ob, V, C = setup(SMALL, seed=6)
    S = int(ob.cluster_offset[1])
    offs = [0, S, S, 2 * S]        # clusters 0 and 2 keep their sources, cluster 1 is empty
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    sky = dd.DeviceSky(t(ob.l[:2 * S]), t(ob.m[:2 * S]), t(ob.I[:2 * S]), t(ob.Q[:2 * S]),
                       t(ob.U[:2 * S]), t(ob.V[:2 * S]), offs)
    obs = dd.device_obs(ob)
    su, sv, sw = dd.device_station_uvw(ob)
    got = dd.unplanes(ctx.predict_factored(obs, su, sv, sw, sky, prec).cpu().numpy())
    tol = 1e-11 if prec == 0 else 1e-5
    assert np.all(got[1] == 0)
    assert rel(got[0], C[0]) <= tol
    assert rel(got[2], C[1]) <= tol


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_factored_vs_direct_full_size(dd, ctx, prec):
    """N=512, K=20 x 50 sources (the bench workload): every coherency of the factorised
    predict against the direct predict on the device, and sampled ones against the oracle."""
    import torch
    cfg = synth.CONFIGS["n512_k20"]
    ob = synth.make_obs(cfg, seed=0, with_noise=False)
    obs, sky = dd.device_obs(ob), dd.device_sky(ob)
    su, sv, sw = dd.device_station_uvw(ob)
    a = ctx.predict_factored(obs, su, sv, sw, sky, prec)
    b = ctx.predict(obs, sky, prec)
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))
    assert err <= (2e-11 if prec == 0 else 2e-5), err
    # sampled visibilities of every cluster against the oracle's per-visibility sum
    rng = np.random.default_rng(7)
    idx = rng.integers(0, ob.B, 64)
    t = int(rng.integers(0, ob.T))
    sub = slice(None)
    ref = rime.predict(ob.u[t:t + 1, idx], ob.v[t:t + 1, idx], ob.w[t:t + 1, idx], ob.freqs,
                       ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, ob.cluster_offset)
    got = dd.unplanes(a[:, :, t:t + 1, :, :][..., torch.as_tensor(idx, device="cuda")].cpu().numpy())
    tol = 1e-11 if prec == 0 else 1e-5
    assert rel(got, ref) <= tol, rel(got, ref)
    del a, b
    torch.cuda.empty_cache()
