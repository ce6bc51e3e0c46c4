"""Pins of the oracle's damped solve, Levenberg-Marquardt and SAGE sweep."""
import math

import numpy as np
import pytest
from scipy.linalg import solve

from oracle import rime, normal_eq as ne, lm, align
from paper_1910_13908_amd import synth


def test_damped_solve_backward_error_and_lapack():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(40, 64))
    H = A.T @ A                         # PSD with a 24-dimensional null space
    g = rng.normal(size=64)
    mu = 1e-3 * np.max(np.diag(H))
    d = lm.damped_solve(H, g, mu)
    M = H + mu * np.eye(64)
    assert np.linalg.norm(M @ d - g) <= 1e-13 * np.linalg.norm(M) * np.linalg.norm(d)
    assert np.allclose(d, solve(M, g, assume_a="pos"), rtol=1e-10, atol=0)
    # a non-PD matrix reports failure
    assert lm.damped_solve(-H, g, 0.0) is None


def _problem(N=8, K=1, S=4, T=4, F=1, seed=0, noise=True, amp=0.1):
    cfg = synth.ObsConfig(N, K, S, T, tuple(np.linspace(140e6, 160e6, F)) if F > 1 else (150e6,),
                          jones_amp=amp)
    ob = synth.make_obs(cfg, seed=seed, with_noise=noise)
    V, C = rime.make_vis(ob)
    return ob, V, C


def test_noiseless_exact_recovery_single_cluster():
    ob, V, C = _problem(N=10, T=4, noise=False, seed=1)
    J0 = synth.identity_jones(1, ob.N)[0]
    J, info = lm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=40)
    assert align.align_error(J, ob.jones_true[0]) <= 1e-10
    assert info.cost <= 1e-20 * rime.cost(V)


def test_accepted_costs_never_increase_and_resume_is_exact():
    ob, V, C = _problem(N=8, T=3, seed=2)
    J0 = synth.identity_jones(1, ob.N)[0]
    J20, i20 = lm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=20)
    c = [i20.cost0] + i20.costs
    assert all(b <= a for a, b in zip(c, c[1:]))
    assert i20.n_accept + i20.n_reject == 20 and i20.n_accept >= 5
    # 10 + 10 iterations with (mu, nu) carried over equals 20 iterations
    J10, i10 = lm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=10)
    Jb, ib = lm.lm_solve(V, C[0], J10, ob.ant_p, ob.ant_q, n_iter=10, mu=i10.mu, nu=i10.nu)
    assert np.array_equal(Jb, J20) and ib.cost == i20.cost


def test_rejected_step_updates_damping():
    # a rejection multiplies mu by nu and doubles nu (Madsen-Nielsen-Tingleff)
    ob, V, C = _problem(N=6, T=2, seed=3)
    J0 = synth.identity_jones(1, ob.N)[0]
    H, g, f = ne.normal_equations(V, C[0], J0, ob.ant_p, ob.ant_q)
    mu0 = 1e-3 * np.max(np.diag(H))
    _, info = lm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=1)
    if info.accepted[0]:
        assert info.nu == 2.0 and info.mu <= mu0 * 1.0000001 and info.mu >= mu0 / 3 * 0.9999999
    else:
        assert info.mu == 2 * mu0 and info.nu == 4.0


def test_chi_square_bound_n64():
    # at the optimum with CN(0, s^2) noise, ||r||^2 ~ (s^2/2) chi^2 with 8BTF - (8N - 4) dof
    # (4 = dimension of the unitary gauge of an unpolarised cluster)
    cfg = synth.CONFIGS["n64_k1"]
    ob = synth.make_obs(cfg, seed=0)
    V, C = rime.make_vis(ob)
    J, info = lm.lm_solve(V, C[0], synth.identity_jones(1, 64)[0], ob.ant_p, ob.ant_q, n_iter=20)
    s2 = cfg.sigma_jy ** 2
    BTF = ob.B * ob.T * ob.F
    dof = 8 * BTF - 8 * ob.N + 4
    mean = 0.5 * s2 * dof
    std = 0.5 * s2 * math.sqrt(2 * dof)
    assert abs(mean - 8.0386) < 1e-3
    assert abs(info.cost - mean) <= 4 * std, (info.cost, mean, std)
    # and the planted gains are recovered to the noise level
    assert align.align_error(J, ob.jones_true[0]) < 5e-3


def test_sage_monotone_and_noiseless_convergence():
    # SAGE converges linearly over sweeps (rate set by the coupling between clusters)
    ob, V, C = _problem(N=12, K=2, S=3, T=6, noise=False, seed=4, amp=0.1)
    J0 = synth.identity_jones(2, ob.N)
    J, R, infos, totals = lm.calibrate(V, C, J0, ob.ant_p, ob.ant_q, n_sweeps=20, n_lm=10,
                                       track_total_cost=True)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(totals, totals[1:]))
    assert totals[-1] <= 1e-15 * rime.cost(V)
    for k in range(2):
        assert align.align_error(J[k], ob.jones_true[k]) < 1e-6
