"""Pins of the oracle's predict against closed forms, invariants and 50-digit arithmetic."""
import math

import numpy as np
import pytest

from oracle import rime
from paper_1910_13908_amd import synth

C = rime.C_LIGHT


def _one(u, v, w, f, l, m, I=1.0, Q=0.0, U=0.0, V=0.0):
    a = lambda x: np.atleast_1d(np.asarray(x, dtype=np.float64))
    uu, vv, ww = (np.asarray(x, dtype=np.float64).reshape(1, -1) for x in (u, v, w))
    return rime.predict(uu, vv, ww, a(f), a(l), a(m), a(I), a(Q), a(U), a(V),
                        np.array([0, np.size(l)]))


def test_phase_centre_constant_coherency():
    # a source at the phase centre: C = B_s on every baseline, whatever u, v, w and f
    rng = np.random.default_rng(1)
    u, v, w = rng.normal(0, 5e3, (3, 2, 37))
    Cc = rime.predict(u, v, w, np.array([120e6, 180e6]), np.array([0.0]), np.array([0.0]),
                      np.array([2.5]), np.array([0.3]), np.array([-0.2]), np.array([0.1]),
                      np.array([0, 1]))
    expect = np.array([[2.8, -0.2 + 0.1j], [-0.2 - 0.1j, 2.2]])
    assert np.array_equal(Cc[0], np.broadcast_to(expect, Cc[0].shape))


def test_quarter_turn_sign():
    # u l f / c = 1/4 turn with v = w = 0 and m = 0: factor exp(-i pi/2) = -i exactly
    f = 150e6
    lam = C / f
    l = 0.01
    u = 0.25 * lam / l
    Cc = _one([u], [0.0], [0.0], f, l, 0.0, I=3.0)[0, 0, 0, 0]
    assert abs(Cc[0, 0] - (-3.0j)) < 1e-14
    assert abs(Cc[1, 1] - (-3.0j)) < 1e-14
    assert Cc[0, 1] == 0 and Cc[1, 0] == 0
    # half a turn gives -1, on the opposite sign of u gives +i
    Cc = _one([2 * u, -u], [0.0, 0.0], [0.0, 0.0], f, l, 0.0)[0, 0, 0]
    assert abs(Cc[0, 0, 0] + 1.0) < 1e-14
    assert abs(Cc[1, 0, 0] - 1.0j) < 1e-14


def test_each_channel_takes_its_own_frequency():
    # the phase scales with f: one baseline, a quarter turn at f, so the channels f, 2f, 3f
    # and 4f see -i, -1, +i and +1 (the same u l, four frequencies in one call)
    f = 150e6
    l = 0.01
    u = 0.25 * (C / f) / l
    Cc = _one([u], [0.0], [0.0], [f, 2 * f, 3 * f, 4 * f], l, 0.0)[0, 0, :, 0, 0, 0]
    for got, want in zip(Cc, (-1.0j, -1.0, 1.0j, 1.0)):
        assert abs(got - want) < 1e-13, (got, want)


def test_w_term_zero_at_centre_and_matches_sqrt():
    assert rime.n_minus_1(0.0, 0.0) == 0.0
    import mpmath
    mpmath.mp.dps = 50
    rng = np.random.default_rng(2)
    for l, m in rng.uniform(-0.3, 0.3, (50, 2)):
        ref = mpmath.sqrt(1 - mpmath.mpf(l) ** 2 - mpmath.mpf(m) ** 2) - 1
        got = rime.n_minus_1(l, m)
        assert abs(float((mpmath.mpf(float(got)) - ref) / ref)) < 4e-16


def test_w_only_phase():
    # source with l = m = 0 ignores w; a source at (l, 0) with only w set gives the n-1 phase
    f = 150e6
    l = 0.05
    w = 123.4
    Cc = _one([0.0], [0.0], [w], f, l, 0.0)[0, 0, 0, 0, 0, 0]
    import mpmath
    mpmath.mp.dps = 50
    ph = mpmath.mpf(w) * (mpmath.sqrt(1 - mpmath.mpf(l) ** 2) - 1) * mpmath.mpf(f) / mpmath.mpf(C)
    ref = complex(mpmath.exp(-2j * mpmath.pi * ph))
    assert abs(Cc - ref) < 1e-13


def test_hermitian_symmetry_reversed_baseline():
    # reversing a baseline (uvw -> -uvw) conjugate-transposes the coherency: V_qp = V_pq^H
    cfg = synth.ObsConfig(6, 2, 4, 3, (140e6, 160e6), polarised=True)
    ob = synth.make_obs(cfg, seed=3)
    a = rime.predict(ob.u, ob.v, ob.w, ob.freqs, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, ob.cluster_offset)
    b = rime.predict(-ob.u, -ob.v, -ob.w, ob.freqs, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, ob.cluster_offset)
    assert np.allclose(b, np.conj(np.swapaxes(a, -1, -2)), rtol=0, atol=1e-12)


def test_linearity_and_superposition():
    cfg = synth.ObsConfig(5, 1, 6, 2, (150e6,), polarised=True)
    ob = synth.make_obs(cfg, seed=4)
    args = (ob.u, ob.v, ob.w, ob.freqs)
    full = rime.predict(*args, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, np.array([0, 6]))
    parts = sum(rime.predict(*args, ob.l[i:i + 1], ob.m[i:i + 1], ob.I[i:i + 1], ob.Q[i:i + 1],
                             ob.U[i:i + 1], ob.V[i:i + 1], np.array([0, 1])) for i in range(6))
    assert np.allclose(full, parts, atol=1e-12)
    doubled = rime.predict(*args, ob.l, ob.m, 2 * ob.I, 2 * ob.Q, 2 * ob.U, 2 * ob.V, np.array([0, 6]))
    assert np.allclose(doubled, 2 * full, atol=1e-12)


def test_periodicity_in_u():
    f, l = 150e6, 0.02
    period = C / (f * l)
    a = _one([10.0], [0.0], [0.0], f, l, 0.0)
    b = _one([10.0 + 7 * period], [0.0], [0.0], f, l, 0.0)
    assert np.allclose(a, b, atol=1e-11)


def test_clusters_are_separate():
    cfg = synth.ObsConfig(5, 3, 2, 2, (150e6,))
    ob = synth.make_obs(cfg, seed=5)
    Cc = rime.predict(ob.u, ob.v, ob.w, ob.freqs, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, ob.cluster_offset)
    for k in range(3):
        s = slice(2 * k, 2 * k + 2)
        one = rime.predict(ob.u, ob.v, ob.w, ob.freqs, ob.l[s], ob.m[s], ob.I[s], ob.Q[s], ob.U[s],
                           ob.V[s], np.array([0, 2]))
        assert np.allclose(Cc[k], one[0], atol=1e-13)


def test_fp64_phase_path_against_mpmath_on_longest_baselines():
    # 100 random terms on the longest baselines of the N=512 layout.  The phase reaches a few
    # thousand turns there, so FP64 itself limits the result: a handful of roundings of size
    # eps * |phase| each, i.e. |err| <= 2 pi * 8 eps * sum|terms| turns (about 1e-11 here).
    import mpmath
    mpmath.mp.dps = 50
    cfg = synth.CONFIGS["n512_k20"]
    rng = np.random.default_rng(6)
    enu = synth.stations_enu(cfg, np.random.default_rng(np.random.SeedSequence(0).spawn(5)[0]))
    suvw = synth.station_uvw(cfg, enu)
    p, q = synth.canonical_baselines(cfg.n_stations)
    buvw = suvw[:, p, :] - suvw[:, q, :]
    lens = np.linalg.norm(buvw[0], axis=1)
    longest = np.argsort(lens)[-100:]
    for b in longest:
        t = int(rng.integers(cfg.n_times))
        l, m = rng.uniform(-0.14, 0.14, 2)
        u, v, w = buvw[t, b]
        f = 150e6
        got = _one([u], [v], [w], f, l, m)[0, 0, 0, 0, 0, 0]
        L, M = mpmath.mpf(float(l)), mpmath.mpf(float(m))
        n1 = mpmath.sqrt(1 - L * L - M * M) - 1
        ph = (mpmath.mpf(float(u)) * L + mpmath.mpf(float(v)) * M + mpmath.mpf(float(w)) * n1) * mpmath.mpf(f) / mpmath.mpf(C)
        ref = complex(mpmath.exp(-2j * mpmath.pi * ph))
        mag = (abs(u * l) + abs(v * m) + abs(w * float(n1))) * f / C
        tol = 2 * math.pi * 8 * 2.0 ** -53 * mag + 1e-15
        assert abs(got - ref) < tol, (b, got, ref, tol)
