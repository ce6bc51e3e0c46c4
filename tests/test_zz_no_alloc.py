"""ddc_residual_noalloc (the entry point for callers that cannot allocate) against
ddc_residual, through the C ABI: the same residual planes and cost, bit for bit (same kernels,
same summation order), on two calls in a row with the second smaller, in both precisions;
the context it runs on never grows a workspace; inputs beyond the stated limits are refused
before any work."""
import ctypes as ct

import numpy as np
import pytest

from oracle import rime
from paper_1910_13908_amd import synth

pytestmark = pytest.mark.gpu

CASES = [synth.ObsConfig(40, 3, 4, 3, (140e6, 160e6), jones_amp=0.2),   # B = 780, ragged
         synth.ObsConfig(20, 2, 3, 2, (150e6,), jones_amp=0.1)]         # smaller second call


@pytest.fixture(scope="module")
def dd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1910_13908_amd import ddcal
    return ddcal


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_noalloc_residual_equals_residual(dd, prec):
    import torch
    ref_ctx = dd.Context(0)
    na_ctx = dd.Context(0)
    dt = torch.float64 if prec == dd.FP64 else torch.float32
    try:
        assert na_ctx.workspace_bytes() == 0
        for i, cfg in enumerate(CASES):
            ob = synth.make_obs(cfg, seed=30 + i)
            V, C = rime.make_vis(ob)
            obs, sky = dd.device_obs(ob), dd.device_sky(ob)
            Vd = torch.as_tensor(dd.planes(V), dtype=dt, device="cuda").contiguous()
            coh = ref_ctx.predict(obs, sky, prec)
            rng = np.random.default_rng(i)
            J = ob.jones_true + 0.01 * (rng.normal(size=ob.jones_true.shape)
                                        + 1j * rng.normal(size=ob.jones_true.shape))
            Jd = torch.as_tensor(dd.jones_real(J), device="cuda").contiguous()
            R_ref = torch.empty_like(Vd)
            c_ref = ref_ctx.residual(obs, ob.K, Vd, coh, Jd, prec, res=R_ref)
            R_na = torch.full_like(Vd, float("nan"))
            c_na = na_ctx.residual_noalloc(obs, ob.K, Vd, coh, Jd, prec, res=R_na)
            torch.cuda.synchronize()
            assert torch.equal(R_na, R_ref), i
            assert c_na == c_ref, (i, c_na, c_ref)
            # cost only, and residual only
            assert na_ctx.residual_noalloc(obs, ob.K, Vd, coh, Jd, prec) == c_ref
            R2 = torch.zeros_like(Vd)
            na_ctx.residual_noalloc(obs, ob.K, Vd, coh, Jd, prec, res=R2, want_cost=False)
            torch.cuda.synchronize()
            assert torch.equal(R2, R_ref), i
            assert na_ctx.workspace_bytes() == 0
    finally:
        ref_ctx.close()
        na_ctx.close()


def test_noalloc_limits_are_refused(dd):
    import torch
    ctx = dd.Context(0)
    try:
        x = torch.zeros(16, dtype=torch.float64, device="cuda")
        for N, T in ((513, 1), (512, 129)):
            obs = dd.Obs(N, T, 1, x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr())
            cost = ct.c_double(0.0)
            st = dd._lib.ddc_residual_noalloc(ctx.h, ct.byref(obs), 1, x.data_ptr(), x.data_ptr(),
                                              x.data_ptr(), 0, x.data_ptr(), ct.byref(cost))
            assert st == dd.EINVAL, (N, T, st)
            assert b"no-allocation limit" in dd._lib.ddc_last_error(ctx.h)
        assert ctx.workspace_bytes() == 0
    finally:
        ctx.close()
