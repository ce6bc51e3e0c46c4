"""Pins of the oracle's Jacobian, normal matrix H and right-hand side g."""
import numpy as np

from oracle import rime, normal_eq as ne
from paper_1910_13908_amd import synth


def _setup(polarised=False, noise=True, seed=0, N=4, T=2, F=2):
    cfg = synth.ObsConfig(N, 1, 3, T, tuple(np.linspace(140e6, 160e6, F)), polarised=polarised,
                          jones_amp=0.3)
    ob = synth.make_obs(cfg, seed=seed, with_noise=noise)
    V, C = rime.make_vis(ob)
    return ob, V, C[0]


def _cost_at(x, Y, C, ob):
    return rime.cost(Y - rime.model_cluster(C, ne.unpack_jones(x), ob.ant_p, ob.ant_q))


def test_jacobian_matches_central_differences():
    ob, V, C = _setup(polarised=True)
    rng = np.random.default_rng(1)
    J = ob.jones_true[0] + 0.1 * (rng.normal(size=(4, 2, 2)) + 1j * rng.normal(size=(4, 2, 2)))
    x = ne.pack_jones(J)
    A_p, A_q = ne.jacobian_blocks(C, J[ob.ant_p], J[ob.ant_q])
    h = 1e-6
    for j in range(x.size):
        e = np.zeros_like(x)
        e[j] = h
        dm = (rime.model_cluster(C, ne.unpack_jones(x + e), ob.ant_p, ob.ant_q)
              - rime.model_cluster(C, ne.unpack_jones(x - e), ob.ant_p, ob.ant_q)) / (2 * h)
        fd = ne.to_real8(dm)                         # [T, F, B, 8]
        st, c = divmod(j, 8)
        an = np.zeros_like(fd)
        sel_p = ob.ant_p == st
        sel_q = ob.ant_q == st
        an[:, :, sel_p, :] += A_p[..., c][:, :, sel_p, :]
        an[:, :, sel_q, :] += A_q[..., c][:, :, sel_q, :]
        assert np.max(np.abs(fd - an)) <= 1e-8 * max(1.0, np.max(np.abs(an))), j


def test_g_is_minus_half_gradient_of_cost():
    ob, V, C = _setup(polarised=True, seed=2)
    rng = np.random.default_rng(3)
    J = ob.jones_true[0] + 0.1 * (rng.normal(size=(4, 2, 2)) + 1j * rng.normal(size=(4, 2, 2)))
    H, g, f = ne.normal_equations(V, C, J, ob.ant_p, ob.ant_q)
    x = ne.pack_jones(J)
    assert abs(f - _cost_at(x, V, C, ob)) <= 1e-13 * f
    h = 1e-6
    grad = np.array([(_cost_at(x + h * e, V, C, ob) - _cost_at(x - h * e, V, C, ob)) / (2 * h)
                     for e in np.eye(x.size)])
    assert np.allclose(g, -0.5 * grad, rtol=0, atol=1e-7 * np.max(np.abs(grad)))


def test_H_is_half_hessian_at_zero_residual():
    # with noiseless data at the true gains r = 0, so d2f/dx2 = 2 A^T A exactly
    ob, V, C = _setup(polarised=True, noise=False, seed=4)
    J = ob.jones_true[0]
    H, g, f = ne.normal_equations(V, C, J, ob.ant_p, ob.ant_q)
    assert f < 1e-25 and np.max(np.abs(g)) < 1e-12
    x = ne.pack_jones(J)
    n = x.size
    h = 1e-4
    E = np.eye(n) * h
    Hfd = np.empty((n, n))
    for i in range(n):
        for j in range(i, n):
            v = (_cost_at(x + E[i] + E[j], V, C, ob) - _cost_at(x + E[i] - E[j], V, C, ob)
                 - _cost_at(x - E[i] + E[j], V, C, ob) + _cost_at(x - E[i] - E[j], V, C, ob)) / (4 * h * h)
            Hfd[i, j] = Hfd[j, i] = 0.5 * v
    assert np.max(np.abs(H - Hfd)) <= 1e-6 * np.max(np.abs(H))


def test_H_symmetric_psd_with_gauge_null_space():
    ob, V, C = _setup(noise=True, seed=5)
    rng = np.random.default_rng(6)
    J = ob.jones_true[0] + 0.05 * (rng.normal(size=(4, 2, 2)) + 1j * rng.normal(size=(4, 2, 2)))
    H, g, f = ne.normal_equations(V, C, J, ob.ant_p, ob.ant_q)
    assert np.array_equal(H, H.T)
    ev = np.linalg.eigvalsh(H)
    assert ev[0] > -1e-12 * ev[-1]
    # unpolarised: J_p -> J_p exp(eps Omega), Omega anti-Hermitian, leaves the model unchanged
    basis = [np.array([[1j, 0], [0, 0]]), np.array([[0, 0], [0, 1j]]),
             np.array([[0, 1], [-1, 0]]), np.array([[0, 1j], [1j, 0]])]
    for Om in basis:
        t = ne.pack_jones(J @ Om)
        assert np.linalg.norm(H @ t) <= 1e-12 * np.linalg.norm(H) * np.linalg.norm(t)
    # exactly four (near-)zero eigenvalues
    assert np.sum(ev < 1e-10 * ev[-1]) == 4


def test_polarised_gauge_is_one_dimensional():
    ob, V, C = _setup(polarised=True, noise=True, seed=7)
    J = ob.jones_true[0]
    H, _, _ = ne.normal_equations(V, C, J, ob.ant_p, ob.ant_q)
    t = ne.pack_jones(1j * J)
    assert np.linalg.norm(H @ t) <= 1e-12 * np.linalg.norm(H) * np.linalg.norm(t)
    ev = np.linalg.eigvalsh(H)
    assert np.sum(ev < 1e-10 * ev[-1]) == 1


def _compact(Y, C, J, ant_p, ant_q):
    """Independent derivation of H and g through per-station / per-baseline 2x2 sums.

    With E_i = c_i e_a e_b^T and E_j = c_j e_c e_d^T (c = 1 or i):
      left  (p) diagonal: Re(conj(c_i) c_j [a==c] P_db),  P = sum G G^H
      right (q) diagonal: Re(c_i conj(c_j) [a==c] Q_bd),  Q = sum Hm^H Hm
      cross (p, q):       Re(conj(c_i c_j) S_abcd),       S_abcd = sum conj(G_bc) Hm_ad
      g_p = (Re, Im) of sum R G^H (p left) + sum R^H Hm (p right)
    """
    N = J.shape[0]
    H = np.zeros((8 * N, 8 * N))
    g = np.zeros(8 * N)
    cs = [1.0, 1.0j]
    for b in range(len(ant_p)):
        p, q = int(ant_p[b]), int(ant_q[b])
        Cb = C[:, :, b]
        Gb = Cb @ np.conj(J[q].T)
        Hb = J[p] @ Cb
        Rb = Y[:, :, b] - Hb @ np.conj(J[q].T)
        P = np.einsum("tfij,tfkj->ik", Gb, np.conj(Gb))
        Q = np.einsum("tfji,tfjk->ik", np.conj(Hb), Hb)
        zl = np.einsum("tfij,tfkj->ik", Rb, np.conj(Gb))
        zr = np.einsum("tfji,tfjk->ik", np.conj(Rb), Hb)
        for i in range(8):
            a, bb = divmod(i // 2, 2)
            ci = cs[i % 2]
            for j in range(8):
                c, d = divmod(j // 2, 2)
                cj = cs[j % 2]
                if a == c:
                    H[8 * p + i, 8 * p + j] += (np.conj(ci) * cj * P[d, bb]).real
                    H[8 * q + i, 8 * q + j] += (ci * np.conj(cj) * Q[bb, d]).real
                S = np.sum(np.conj(Gb[:, :, bb, c]) * Hb[:, :, a, d])
                H[8 * p + i, 8 * q + j] += (np.conj(ci * cj) * S).real
                H[8 * q + j, 8 * p + i] += (np.conj(ci * cj) * S).real
        g[8 * p:8 * p + 8] += ne.to_real8(zl)
        g[8 * q:8 * q + 8] += ne.to_real8(zr)
    return H, g


def test_brute_force_equals_compact_form():
    for N, pol in ((3, False), (5, True)):
        ob, V, C = _setup(polarised=pol, seed=8 + N, N=N)
        rng = np.random.default_rng(N)
        J = ob.jones_true[0] + 0.1 * (rng.normal(size=(N, 2, 2)) + 1j * rng.normal(size=(N, 2, 2)))
        H, g, f = ne.normal_equations(V, C, J, ob.ant_p, ob.ant_q)
        Hc, gc = _compact(V, C, J, ob.ant_p, ob.ant_q)
        assert np.allclose(H, Hc, rtol=0, atol=1e-12 * np.max(np.abs(H)))
        assert np.allclose(g, gc, rtol=0, atol=1e-12 * np.max(np.abs(g)))


def test_pack_unpack_layout():
    # x[2e] = Re J_e, x[2e+1] = Im J_e, entries 00, 01, 10, 11
    J1 = np.array([[[1 + 2j, 3 + 4j], [5 + 6j, 7 + 8j]]])
    assert list(ne.pack_jones(J1)) == [1, 2, 3, 4, 5, 6, 7, 8]
    assert np.array_equal(ne.unpack_jones(ne.pack_jones(J1)), J1)
