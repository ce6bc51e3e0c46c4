"""Levenberg-Marquardt on the GPU against the oracle iteration by iteration, and the LM's
failure paths, through the C ABI.

* The per-iteration records of ddc_lm_solve (cost after the iteration, mu_eff, mu, nu,
  accepted) follow the oracle's (Madsen, Nielsen & Tingleff 2004, Algorithm 3.16) on the
  N = 64, one-cluster, 20-iteration FP64 workload, for as long as each accept/reject is
  decided by more than the rounding of the cost sums: the first iteration whose trial
  decrease |f - f'| is below 1e-9 f may go either way (the two sides add the cost in
  different orders), and after it only the results are compared.
* The same trace through ddc_calibrate (a one-sweep calibration of one cluster is one LM).
* A zero Jones start makes H = 0, g = 0 and max diag = 0 (the model is bilinear in the
  Jones), so mu = mu_eff = 0 and the factorisation of the zero matrix fails: every step is
  a rejection counted as a failed factorisation, on both sides, in both precisions.
* NaN in the data makes the cost non-finite: DDC_ENONFINITE from ddc_lm_solve (the Jones
  untouched), ddc_calibrate and ddc_residual.
* With the inter-workgroup waits bounded at one retry (ddc_set_wait_limit), the solves time
  out and the calls report DDC_ETIMEOUT with the Jones untouched; the context then solves
  normally.  Every kernel still leaves normally: the bound only makes waits give up sooner.
* Calls that put their own buffers in the context's workspace (the residual, the cost
  gradient) between two solves leave the later solve bit-identical to a fresh context's,
  with N = 10 (matrix storage padded from 80 to 128 rows).
"""
import math

import numpy as np
import pytest

from oracle import lm as olm, align
from paper_1910_13908_amd import synth

from _gpu_util import setup, to_dev

pytestmark = pytest.mark.gpu

CFG64 = synth.CONFIGS["n64_k1"]


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


@pytest.fixture(scope="module")
def n64():
    ob, V, C = setup(CFG64, seed=0)
    J0 = synth.identity_jones(1, ob.N)[0]
    Jo, io = olm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=CFG64.n_lm)
    return ob, V, C, J0, Jo, io


def _determined_prefix(io, rel=1e-9):
    """Iterations [0, n) whose accept/reject is decided above the rounding level: up to and
    including the first one whose trial decrease is below rel * f."""
    f_before = [io.cost0] + list(io.costs[:-1])
    for i, (fb, ft) in enumerate(zip(f_before, io.trial_costs)):
        if math.isfinite(ft) and abs(fb - ft) <= rel * fb:
            return i
    return len(io.costs)


def _compare_trace(tr, io, n_det, cost_tol):
    assert n_det >= 3, n_det                     # the comparison covers the descent
    for i in range(n_det):
        s = tr[i]
        assert bool(s.accepted) == io.accepted[i], (i, s.accepted, io.accepted[i])
        assert abs(s.cost - io.costs[i]) <= cost_tol * io.costs[i], (i, s.cost, io.costs[i])
        for got, ref in ((s.mu_eff, io.mu_effs[i]), (s.mu, io.mus[i])):
            assert abs(got - ref) <= 1e-8 * ref, (i, got, ref)
        assert s.nu == io.nus[i], (i, s.nu, io.nus[i])


def test_lm_trace_fp64_follows_oracle(dd, ctx, n64):
    import torch
    ob, V, C, J0, Jo, io = n64
    d = to_dev(dd, ob, dd.FP64, V=V)
    coh = ctx.predict(d["obs"], d["sky"], dd.FP64)[0].contiguous()
    Jd = torch.as_tensor(dd.jones_real(J0), device="cuda").contiguous()
    opts = dd.default_lm_opts(n_iter=CFG64.n_lm, precision=dd.FP64)
    info, tr = ctx.lm_solve(d["obs"], d["V"], coh, Jd, opts, want_trace=True)
    assert len(tr) == CFG64.n_lm
    n_det = _determined_prefix(io)
    _compare_trace(tr, io, n_det, 1e-9)
    # the counts and the last record agree with the report
    assert info.n_accept == sum(s.accepted for s in tr)
    assert info.n_accept + info.n_reject == CFG64.n_lm
    assert tr[-1].cost == info.cost
    # every record after the determined prefix still sits at the oracle's cost
    for i in range(n_det, CFG64.n_lm):
        assert abs(tr[i].cost - io.costs[i]) <= 1e-8 * io.costs[i], i
    assert align.align_error(dd.jones_complex(Jd.cpu().numpy()), Jo) <= 1e-8


def test_lm_trace_mixed_against_oracle(dd, ctx, n64):
    # mixed: FP32 normal equations, FP64 cost and refinement; the descent takes the same
    # decisions and its costs agree to the mixed tolerance
    import torch
    ob, V, C, J0, Jo, io = n64
    d = to_dev(dd, ob, dd.MIXED, V=V)
    coh = ctx.predict(d["obs"], d["sky"], dd.MIXED)[0].contiguous()
    Jd = torch.as_tensor(dd.jones_real(J0), device="cuda").contiguous()
    opts = dd.default_lm_opts(n_iter=CFG64.n_lm, precision=dd.MIXED)
    info, tr = ctx.lm_solve(d["obs"], d["V"], coh, Jd, opts, want_trace=True)
    n_det = _determined_prefix(io, rel=1e-5)
    for i in range(n_det):
        assert bool(tr[i].accepted) == io.accepted[i], i
        assert abs(tr[i].cost - io.costs[i]) <= 1e-5 * io.costs[i], (i, tr[i].cost, io.costs[i])
    assert abs(info.cost - io.cost) <= 1e-5 * io.cost
    assert align.align_error(dd.jones_complex(Jd.cpu().numpy()), Jo) <= 1e-4
    assert all(s.refine_steps >= 1 for s in tr if s.accepted)


def test_calibrate_trace_is_the_lm_trace(dd, ctx, n64):
    import torch
    ob, V, C, J0, Jo, io = n64
    d = to_dev(dd, ob, dd.FP64, V=V)
    Jd = torch.as_tensor(dd.jones_real(synth.identity_jones(1, ob.N)), device="cuda").contiguous()
    opts = dd.default_lm_opts(n_iter=CFG64.n_lm, precision=dd.FP64)
    infos, tr = ctx.calibrate(d["obs"], d["sky"], d["V"], Jd, 1, opts, want_trace=True)
    tr = tr[0][0]
    _compare_trace(tr, io, _determined_prefix(io), 1e-9)
    assert tr[-1].cost == infos[0][0].cost


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_failed_factorisation_is_a_rejection(dd, ctx, prec):
    import torch
    cfg = synth.ObsConfig(12, 1, 4, 3, (150e6,))
    ob, V, C = setup(cfg, seed=4)
    J0 = np.zeros((ob.N, 2, 2), dtype=np.complex128)
    Jo, io = olm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=3)
    assert io.n_notpd == 3 and io.n_accept == 0       # the oracle's reading of this case
    d = to_dev(dd, ob, prec, V=V)
    coh = ctx.predict(d["obs"], d["sky"], prec)[0].contiguous()
    Jd = torch.zeros((ob.N, 8), dtype=torch.float64, device="cuda")
    info, tr = ctx.lm_solve(d["obs"], d["V"], coh, Jd, dd.default_lm_opts(n_iter=3, precision=prec),
                            want_trace=True)
    assert (info.n_notpd, info.n_reject, info.n_accept) == (3, 3, 0)
    assert not torch.any(Jd != 0)
    assert [s.accepted for s in tr] == [0, 0, 0]
    assert [s.nu for s in tr] == io.nus
    assert [s.mu for s in tr] == io.mus == [0.0, 0.0, 0.0]
    assert abs(info.cost - io.cost) <= (1e-12 if prec == 0 else 1e-6) * io.cost


def test_nonfinite_data_is_reported(dd, ctx):
    import torch
    cfg = synth.ObsConfig(10, 2, 3, 2, (150e6,))
    ob, V, C = setup(cfg, seed=5)
    for prec in (dd.FP64, dd.MIXED):
        d = to_dev(dd, ob, prec, V=V)
        Vbad = d["V"].clone()
        Vbad[3, 1, 0, 7] = float("nan")
        coh = ctx.predict(d["obs"], d["sky"], prec)
        J = torch.as_tensor(dd.jones_real(synth.identity_jones(2, ob.N)), device="cuda").contiguous()
        J0 = J.clone()
        with pytest.raises(dd.DdcError) as e:
            ctx.lm_solve(d["obs"], Vbad, coh[0].contiguous(), J[0], dd.default_lm_opts(n_iter=2, precision=prec),
                         want_info=False)
        assert e.value.status == dd.ENONFINITE
        assert torch.equal(J, J0)
        with pytest.raises(dd.DdcError) as e:
            ctx.calibrate(d["obs"], d["sky"], Vbad, J, 1, dd.default_lm_opts(n_iter=2, precision=prec),
                          want_info=False)
        assert e.value.status == dd.ENONFINITE
        with pytest.raises(dd.DdcError) as e:
            ctx.residual(d["obs"], 2, Vbad, coh, J0, prec)
        assert e.value.status == dd.ENONFINITE
        # the clean data still solve on the same context afterwards
        J = J0.clone()
        info = ctx.lm_solve(d["obs"], d["V"], coh[0].contiguous(), J[0], dd.default_lm_opts(n_iter=2, precision=prec))
        assert info.n_accept >= 1


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_wait_timeout_is_reported_and_the_context_recovers(dd, n64, prec):
    # With every inter-workgroup wait bounded at one retry, the factorisation and the solves
    # give up on the first tile or block that is not ready at once: they abort (every
    # workgroup leaves), the step is rejected, and the call reports DDC_ETIMEOUT without an
    # info struct, with the Jones untouched.  The same context then solves normally.
    import torch
    ob, V, C, J0, Jo, io = n64
    ctx = dd.Context(0)
    try:
        d = to_dev(dd, ob, prec, V=V)
        coh = ctx.predict(d["obs"], d["sky"], prec)[0].contiguous()
        J = torch.as_tensor(dd.jones_real(J0), device="cuda").contiguous()
        J_start = J.clone()
        ctx.set_wait_limit(1)
        with pytest.raises(dd.DdcError) as e:
            ctx.lm_solve(d["obs"], d["V"], coh, J, dd.default_lm_opts(n_iter=3, precision=prec),
                         want_info=False)
        assert e.value.status == dd.ETIMEOUT
        assert torch.equal(J, J_start)
        n = 8 * ob.N
        H = torch.eye(n, dtype=torch.float64 if prec == 0 else torch.float32, device="cuda") * 4.0
        g = torch.ones(n, dtype=H.dtype, device="cuda")
        with pytest.raises(dd.DdcError) as e:
            ctx.damped_solve(H, g, 0.0, prec)
        assert e.value.status == dd.ETIMEOUT
        ctx.set_wait_limit(0)
        info = ctx.lm_solve(d["obs"], d["V"], coh, J, dd.default_lm_opts(n_iter=CFG64.n_lm, precision=prec))
        err = align.align_error(dd.jones_complex(J.cpu().numpy()), Jo)
        assert err <= (1e-8 if prec == 0 else 1e-4), err
        assert abs(info.cost - io.cost) <= (1e-9 if prec == 0 else 1e-5) * io.cost
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_other_calls_between_solves_leave_them_unchanged(dd, prec):
    # The residual (with its Jones planes) and the cost gradient use the context's workspace
    # for their own buffers, over the matrix storage whose zeros and padding diagonal a solve
    # writes once.  With N = 10 (8N = 80 rows padded to 128) a later solve on the same context
    # must still equal, bit for bit, the same solve on a fresh context.
    import torch
    cfg = synth.ObsConfig(10, 2, 3, 2, (150e6,))
    ob, V, C = setup(cfg, seed=7)
    a, b = dd.Context(0), dd.Context(0)
    try:
        d = to_dev(dd, ob, prec, V=V)
        coh = a.predict(d["obs"], d["sky"], prec)
        J0 = torch.as_tensor(dd.jones_real(synth.identity_jones(2, ob.N)), device="cuda").contiguous()
        opts = dd.default_lm_opts(n_iter=4, precision=prec)
        Ja = J0.clone()
        ia = a.lm_solve(d["obs"], d["V"], coh[0].contiguous(), Ja[0], opts)
        Jb = J0.clone()
        b.lm_solve(d["obs"], d["V"], coh[0].contiguous(), Jb[0], opts)
        b.residual(d["obs"], 2, d["V"], coh, J0, prec, want_cost=False)
        b.cost_gradient(d["obs"], 2, d["V"], coh, J0, prec)
        Jb = J0.clone()
        ib = b.lm_solve(d["obs"], d["V"], coh[0].contiguous(), Jb[0], opts)
        torch.cuda.synchronize()
        assert ia.n_accept >= 1
        assert (ib.n_accept, ib.n_reject) == (ia.n_accept, ia.n_reject)
        assert ib.cost == ia.cost
        assert torch.equal(Ja, Jb)
    finally:
        a.close()
        b.close()
