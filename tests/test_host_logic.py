"""Host logic of the C ABI that runs without a GPU: every entry point rejects a missing
handle before any device call, the server rejects bad limits before creating anything, and
the workspace footprint of a calibration covers the buffers the method needs."""
import ctypes as ct

import pytest

from paper_1910_13908_amd import ddcal as dd

L = dd._lib
EINVAL = -1


def _obs(N=512, T=10, F=1):
    o = dd.Obs()
    o.n_stations, o.n_times, o.n_chans = N, T, F
    return o


def test_every_entry_point_rejects_a_null_handle():
    o = ct.byref(_obs())
    opts = dd.LMOpts()
    L.ddc_default_lm_opts(ct.byref(opts))
    calls = {
        "ddc_destroy": lambda: L.ddc_destroy(None),
        "ddc_set_stream": lambda: L.ddc_set_stream(None, None),
        "ddc_predict": lambda: L.ddc_predict(None, o, None, 1, None),
        "ddc_predict_factored": lambda: L.ddc_predict_factored(None, o, None, None, None, None, 1, None),
        "ddc_residual": lambda: L.ddc_residual(None, o, 2, None, None, None, 1, None, None),
        "ddc_residual_noalloc": lambda: L.ddc_residual_noalloc(None, o, 2, None, None, None, 1, None, None),
        "ddc_add_model": lambda: L.ddc_add_model(None, o, 2, None, None, None, -1.0, 1, None),
        "ddc_build_normal_eq": lambda: L.ddc_build_normal_eq(None, o, None, None, None, 1, None, None, None),
        "ddc_damped_solve": lambda: L.ddc_damped_solve(None, 64, None, None, 0.0, 1, 1e-10, 5, None, None),
        "ddc_lm_solve": lambda: L.ddc_lm_solve(None, o, None, None, None, ct.byref(opts), None, None, None),
        "ddc_calibrate": lambda: L.ddc_calibrate(None, o, None, None, None, None, None, None, None),
        "ddc_cost_gradient": lambda: L.ddc_cost_gradient(None, o, 2, None, None, None, 1, None, None),
        "ddc_set_wait_limit": lambda: L.ddc_set_wait_limit(None, 0),
        "ddc_enable_timing": lambda: L.ddc_enable_timing(None, 1),
        "ddc_enable_timers": lambda: L.ddc_enable_timers(None, 0),
        "ddc_get_timing": lambda: L.ddc_get_timing(None, 0, None, None, None),
        "ddc_server_destroy": lambda: L.ddc_server_destroy(None),
        "ddc_server_submit": lambda: L.ddc_server_submit(None, o, None, None, None, None, None),
        "ddc_server_wait": lambda: L.ddc_server_wait(None, 0, None, None, None),
        "ddc_server_stats": lambda: L.ddc_server_stats(None, None, None, None),
    }
    bad = {name: st for name, st in ((n, f()) for n, f in calls.items()) if st != EINVAL}
    assert not bad, bad
    assert L.ddc_last_error(None) == b"null context"
    assert L.ddc_server_last_error(None) == b"null server"
    assert L.ddc_workspace_bytes(None) == 0


@pytest.mark.parametrize("n_slots, budget", [(0, 1 << 30), (65, 1 << 30), (4, 1 << 15)])
def test_server_limits_are_checked_first(n_slots, budget):
    h = ct.c_void_p()
    assert L.ddc_server_create(ct.byref(h), 0, n_slots, budget) == EINVAL
    assert not h.value
    assert L.ddc_server_create(None, 0, 4, 1 << 30) == EINVAL


def _fp(o, K=20, sweeps=3, iters=10, prec=dd.MIXED):
    return L.ddc_calibrate_footprint(ct.byref(o) if o is not None else None, K, sweeps, iters, prec)


def test_footprint_rejects_invalid_problems():
    assert _fp(None) == -1
    for N, T, F in ((1, 10, 1), (512, 0, 1), (512, 10, 0)):
        assert _fp(_obs(N, T, F)) == -1
    o = _obs()
    assert _fp(o, K=0) == -1 and _fp(o, sweeps=-1) == -1 and _fp(o, iters=-1) == -1
    assert _fp(o, prec=2) == -1


def _named_buffers(N, T, F, K, es):
    # the buffers a calibration cannot do without: K coherency planes, the residual and one
    # cluster's data (8 planes each), the 8N x 8N matrix, the factor's lower tiles and their
    # transposed copies, the diagonal inverses and their copies, and the 8-byte tagged copies
    # of the lower tiles that the factorisation's tasks read
    B = N * (N - 1) // 2
    plane = T * F * B
    n_pad = (8 * N + 63) // 64 * 64
    t = n_pad // 64
    tiles = t * (t + 1) // 2
    return ((K + 2) * 8 * plane * es + n_pad * n_pad * es + 2 * tiles * 4096 * es
            + 2 * t * 4096 * es + tiles * 4096 * 8)


@pytest.mark.parametrize("N, T, F, K", [(512, 10, 1, 20), (128, 10, 4, 10), (10, 3, 2, 2)])
def test_footprint_covers_the_buffers_the_method_needs(N, T, F, K):
    for prec, es in ((dd.MIXED, 4), (dd.FP64, 8)):
        need = _named_buffers(N, T, F, K, es)
        got = _fp(_obs(N, T, F), K=K, prec=prec)
        assert need <= got <= 1.25 * need + (1 << 20), (prec, need, got)


def test_footprint_grows_by_one_clusters_planes_per_cluster():
    o = _obs()
    plane = 10 * 1 * (512 * 511 // 2)
    for prec, es in ((dd.MIXED, 4), (dd.FP64, 8)):
        d = _fp(o, K=21, prec=prec) - _fp(o, K=20, prec=prec)
        assert 8 * plane * es <= d <= 8 * plane * es + (64 << 10), (prec, d)
    # FP64 stores every element of the planes and matrices at twice the size
    assert _fp(o, prec=dd.FP64) - _fp(o, prec=dd.MIXED) >= _named_buffers(512, 10, 1, 20, 4) - (
        2080 * 4096 * 8)
