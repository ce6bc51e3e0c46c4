"""Pins of the oracle's model, residual, cost and alignment."""
import numpy as np

from oracle import rime, align
from paper_1910_13908_amd import synth


def _tiny(polarised=False, K=1, seed=0, noise=False):
    cfg = synth.ObsConfig(4, K, 3, 2, (140e6, 160e6), polarised=polarised, jones_amp=0.3)
    ob = synth.make_obs(cfg, seed=seed, with_noise=noise)
    C = rime.predict(ob.u, ob.v, ob.w, ob.freqs, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, ob.cluster_offset)
    return ob, C


def test_model_matches_scalar_loops():
    # brute force: M[i][l] = sum_j sum_k Jp[i][j] C[j][k] conj(Jq[l][k]), pure Python scalars
    ob, C = _tiny(polarised=True, K=2)
    J = ob.jones_true
    M = rime.model(C, J, ob.ant_p, ob.ant_q)
    T, F, B = C.shape[1:4]
    for t in range(T):
        for f in range(F):
            for b in range(B):
                p, q = int(ob.ant_p[b]), int(ob.ant_q[b])
                for i in range(2):
                    for l in range(2):
                        acc = 0j
                        for k in range(C.shape[0]):
                            for j in range(2):
                                for kk in range(2):
                                    acc += complex(J[k, p, i, j]) * complex(C[k, t, f, b, j, kk]) * complex(J[k, q, l, kk]).conjugate()
                        assert abs(acc - M[t, f, b, i, l]) < 1e-13


def test_model_hermitian_under_baseline_reversal():
    # V_qp = V_pq^H: swap stations and use C^H (the reversed-baseline coherency)
    ob, C = _tiny(polarised=True)
    J = ob.jones_true
    M = rime.model_cluster(C[0], J[0], ob.ant_p, ob.ant_q)
    Mr = rime.model_cluster(np.conj(np.swapaxes(C[0], -1, -2)), J[0], ob.ant_q, ob.ant_p)
    assert np.allclose(Mr, np.conj(np.swapaxes(M, -1, -2)), atol=1e-13)


def test_noiseless_residual_vanishes():
    ob, C = _tiny(K=2)
    V, _ = rime.make_vis(ob)
    R = rime.residual(V, C, ob.jones_true, ob.ant_p, ob.ant_q)
    assert np.linalg.norm(R) <= 1e-13 * np.linalg.norm(V)
    assert rime.cost(R) <= 1e-26 * rime.cost(V)


def test_cost_is_sum_of_squared_moduli():
    R = np.array([[[[[3 + 4j, 0], [1j, -2]]]]])
    assert rime.cost(R) == 25 + 1 + 4


def _unitary(rng):
    Z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    Q, Rr = np.linalg.qr(Z)
    return Q * (np.diag(Rr) / np.abs(np.diag(Rr)))


def test_cost_invariant_under_unitary_gauge_unpolarised():
    ob, C = _tiny(noise=True, seed=3)
    V, _ = rime.make_vis(ob)
    rng = np.random.default_rng(7)
    J = ob.jones_true + 0.05 * (rng.normal(size=ob.jones_true.shape) + 1j * rng.normal(size=ob.jones_true.shape))
    U = _unitary(rng)
    f1 = rime.cost(rime.residual(V, C, J, ob.ant_p, ob.ant_q))
    f2 = rime.cost(rime.residual(V, C, J @ U, ob.ant_p, ob.ant_q))
    assert abs(f1 - f2) <= 1e-12 * f1
    # ... and not under a non-unitary change
    f3 = rime.cost(rime.residual(V, C, J @ (1.01 * U), ob.ant_p, ob.ant_q))
    assert abs(f3 - f1) > 1e-6 * f1


def test_cost_invariant_under_common_phase_polarised():
    ob, C = _tiny(polarised=True, noise=True, seed=4)
    V, _ = rime.make_vis(ob)
    J = ob.jones_true * 1.02
    f1 = rime.cost(rime.residual(V, C, J, ob.ant_p, ob.ant_q))
    f2 = rime.cost(rime.residual(V, C, J * np.exp(0.7j), ob.ant_p, ob.ant_q))
    assert abs(f1 - f2) <= 1e-12 * f1
    # a general unitary changes the cost when the cluster is polarised
    U = _unitary(np.random.default_rng(8))
    f3 = rime.cost(rime.residual(V, C, J @ U, ob.ant_p, ob.ant_q))
    assert abs(f3 - f1) > 1e-6 * f1


def test_procrustes_recovers_known_unitary():
    rng = np.random.default_rng(9)
    Jref = rng.normal(size=(7, 2, 2)) + 1j * rng.normal(size=(7, 2, 2))
    U = _unitary(rng)
    J = Jref @ np.conj(U.T)
    assert np.allclose(align.procrustes_unitary(J, Jref), U, atol=1e-12)
    assert align.align_error(J, Jref) < 1e-14
    Jp = Jref * np.exp(-1.1j)
    assert align.align_error(Jp, Jref, polarised=True) < 1e-14
    # a non-unitary distortion is not removed
    assert align.align_error(J * 1.1, Jref) > 0.05


def test_synth_shapes_and_baseline_order():
    cfg = synth.CONFIGS["n64_k1"]
    ob = synth.make_obs(cfg, seed=0)
    assert ob.B == 2016 and ob.u.shape == (10, 2016)
    b = 0
    for p in range(64):
        for q in range(p + 1, 64):
            assert ob.ant_p[b] == p and ob.ant_q[b] == q
            b += 1
    # seeds fix everything
    ob2 = synth.make_obs(cfg, seed=0)
    assert np.array_equal(ob.noise, ob2.noise) and np.array_equal(ob.l, ob2.l)
    # station uvw at H = 0 with dec = lat gives (E, N, Up)
    c2 = synth.ObsConfig(3, 1, 1, 1, (150e6,), dec_deg=40.0, lat_deg=40.0)
    enu = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0], [-5.0, 4.0, 0.5]])
    uvw = synth.station_uvw(c2, enu)[0]
    assert np.allclose(uvw, enu, atol=1e-12)
