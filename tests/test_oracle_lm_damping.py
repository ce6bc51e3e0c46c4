"""Pins of the oracle's Levenberg-Marquardt damping schedule, each value recomputed by a route
that shares nothing with ``oracle.lm`` beyond the model itself.

Madsen, Nielsen & Tingleff (2004), Algorithm 3.16, with Levenberg damping mu*I, for
f(x) = ||r(x)||^2 (no factor 1/2):

* fresh start: mu_0 = tau * max diag(A^T A), nu = 2;
* the step solves min ||r - A d||^2 + mu_eff ||d||^2 with mu_eff = max(mu, mu_floor * max diag);
* gain ratio rho = (f(x) - f(x + d)) / (||r||^2 - ||r - A d||^2), the actual decrease over the
  decrease of the linear model;
* rho > 0: accept, mu <- mu * max(1/3, 1 - (2 rho - 1)^3), nu <- 2;
  otherwise mu <- mu * nu, nu <- 2 nu.

Here the Jacobian A is formed by central differences of the model (exact up to rounding: the
model of a baseline is affine in any single real parameter of one station, since no baseline
joins a station to itself), the step by an augmented least-squares solve, and the predicted
decrease as ||r||^2 - ||r - A d||^2 rather than the oracle's d . (mu d + g), which equals it only
when the step solves the damped normal equations.  Each problem is chosen so that the quantity
under test moves the result (a gain ratio well inside (0, 0.9), a small positive one, a
clamped update, a genuine cost increase), so a dropped term, a square for the cube, a halved
denominator, a raised acceptance threshold, a missing doubling of nu or a moved floor each
fail a test.
"""
import numpy as np
import pytest

from oracle import rime, lm, normal_eq as ne
from paper_1910_13908_amd import synth


def _problem(amp, seed, N=5, S=3, T=2):
    cfg = synth.ObsConfig(N, 1, S, T, (150e6,), jones_amp=amp)
    ob = synth.make_obs(cfg, seed=seed)
    V, C = rime.make_vis(ob)
    return ob, V, C[0]


def _flat(M):
    """complex [..., 2, 2] -> real vector (any fixed order; A and r share it)."""
    return np.ascontiguousarray(M).view(np.float64).reshape(-1)


def _x_to_J(x):
    return x.reshape(-1, 4, 2).view(np.complex128)[..., 0].reshape(-1, 2, 2)


def _J_to_x(J):
    return np.ascontiguousarray(J, dtype=np.complex128).view(np.float64).reshape(-1).copy()


def _model(C, x, ob):
    return rime.model_cluster(C, _x_to_J(x), ob.ant_p, ob.ant_q)


def _jacobian_fd(C, x, ob):
    n = x.size
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append((_flat(_model(C, x + e, ob)) - _flat(_model(C, x - e, ob))) / 2.0)
    return np.stack(cols, axis=1)


def _step(A, r, mu):
    """argmin ||r - A d||^2 + mu ||d||^2 by least squares on the stacked system."""
    n = A.shape[1]
    Aa = np.vstack([A, np.sqrt(mu) * np.eye(n)])
    ra = np.concatenate([r, np.zeros(n)])
    return np.linalg.lstsq(Aa, ra, rcond=None)[0]


def _setup(amp, seed):
    ob, V, C = _problem(amp, seed)
    x0 = _J_to_x(synth.identity_jones(1, ob.N)[0])
    r = _flat(V - _model(C, x0, ob))
    A = _jacobian_fd(C, x0, ob)
    return ob, V, C, x0, r, A


def _gain_ratio(ob, V, C, x0, r, A, mu_eff):
    d = _step(A, r, mu_eff)
    f = float(r @ r)
    f_new = rime.cost(V - _model(C, x0 + d, ob))
    pred = f - float(np.sum((r - A @ d) ** 2))
    return d, f, f_new, (f - f_new) / pred


def test_jacobian_by_differences_matches_model_linearisation():
    # the finite-difference Jacobian is the Gauss-Newton one: A^T A is the oracle's H up to a
    # permutation-free reordering of residual rows, so its diagonal and A^T r match
    ob, V, C, x0, r, A = _setup(0.8, 0)
    H, g, f = ne.normal_equations(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q)
    assert np.allclose(A.T @ A, H, rtol=0, atol=1e-10 * np.abs(H).max())
    assert np.allclose(A.T @ r, g, rtol=0, atol=1e-10 * np.abs(g).max())
    assert abs(float(r @ r) - f) <= 1e-13 * f


def test_fresh_start_mu0_is_tau_times_max_diagonal():
    ob, V, C, x0, r, A = _setup(0.8, 0)
    md = float(np.max(np.sum(A * A, axis=0)))
    for tau in (1e-3, 0.25):
        _, info = lm.lm_solve(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q, n_iter=0, tau=tau)
        assert abs(info.mu - tau * md) <= 1e-12 * tau * md
        assert info.nu == 2.0


def test_gain_ratio_and_accepted_damping_update():
    # rho near 0.38 here: unclamped for rho and for 2 rho, and 2 rho - 1 < 0, so the cube and
    # the square of (2 rho - 1) move mu in opposite directions
    ob, V, C, x0, r, A = _setup(0.8, 0)
    md = float(np.max(np.sum(A * A, axis=0)))
    mu = 1e-3 * md
    d, f, f_new, rho = _gain_ratio(ob, V, C, x0, r, A, mu)
    assert 0.2 < rho < 0.45, rho
    J1, info = lm.lm_solve(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q, n_iter=1, mu=mu, nu=2.0)
    assert info.accepted == [True]
    assert np.max(np.abs(_J_to_x(J1) - (x0 + d))) <= 1e-9 * np.max(np.abs(d))
    assert abs(info.cost - f_new) <= 1e-12 * f_new
    expect = mu * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
    assert abs(info.mu - expect) <= 1e-9 * expect, (info.mu, expect)
    assert info.mu > mu                       # rho < 1/2 raises the damping
    assert info.nu == 2.0


def test_small_positive_gain_ratio_is_accepted():
    # any rho > 0 accepts the step (the cost went down, if by less than the linear model
    # promised): here rho is about 0.07, and the update raises mu by 1 - (2 rho - 1)^3
    ob, V, C, x0, r, A = _setup(1.2, 4)
    md = float(np.max(np.sum(A * A, axis=0)))
    mu = 1e-3 * md
    d, f, f_new, rho = _gain_ratio(ob, V, C, x0, r, A, mu)
    assert 0.0 < rho < 0.15, rho
    J1, info = lm.lm_solve(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q, n_iter=1, mu=mu, nu=4.0)
    assert info.accepted == [True]
    assert np.max(np.abs(_J_to_x(J1) - (x0 + d))) <= 1e-9 * np.max(np.abs(d))
    expect = mu * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
    assert abs(info.mu - expect) <= 1e-8 * expect, (info.mu, expect)
    assert info.nu == 2.0


def test_good_step_divides_mu_by_three():
    # rho ~ 1: 1 - (2 rho - 1)^3 < 1/3, so the update takes the clamp
    ob, V, C, x0, r, A = _setup(0.3, 0)
    md = float(np.max(np.sum(A * A, axis=0)))
    mu = 1e-3 * md
    _, _, _, rho = _gain_ratio(ob, V, C, x0, r, A, mu)
    assert rho > 0.95, rho
    _, info = lm.lm_solve(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q, n_iter=1, mu=mu, nu=8.0)
    assert info.accepted == [True]
    assert abs(info.mu - mu / 3.0) <= 1e-15 * mu
    assert info.nu == 2.0                     # an accept resets nu whatever it was


def test_consecutive_rejections_multiply_mu_by_growing_nu():
    # a strongly non-linear start: the damped Gauss-Newton steps raise the cost, so each is
    # rejected; the k-th rejection multiplies mu by 2^k and doubles nu
    ob, V, C, x0, r, A = _setup(1.5, 1)
    md = float(np.max(np.sum(A * A, axis=0)))
    tau = 1e-6
    mu, nu = tau * md, 2.0
    for k in range(1, 4):
        mu_eff = max(mu, 1e-6 * md)
        d, f, f_new, rho = _gain_ratio(ob, V, C, x0, r, A, mu_eff)
        assert f_new > f                      # a genuine increase, independently evaluated
        mu, nu = mu * nu, 2.0 * nu
        J, info = lm.lm_solve(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q, n_iter=k, tau=tau)
        assert info.accepted == [False] * k
        assert np.array_equal(_J_to_x(J), x0)
        assert info.nu == nu == 2.0 ** (k + 1)
        assert abs(info.mu - tau * md * 2.0 ** (k * (k + 1) // 2)) <= 1e-12 * info.mu
        assert abs(info.mu - mu) <= 1e-12 * mu


def test_zero_step_is_rejected():
    # at J = 0 the Jacobian vanishes (the model is bilinear), so g = 0, d = 0 and the predicted
    # decrease is 0: a rejection (rho needs a positive denominator)
    ob, V, C, x0, r, A = _setup(0.3, 2)
    J0 = np.zeros((ob.N, 2, 2), dtype=np.complex128)
    J, info = lm.lm_solve(V, C, J0, ob.ant_p, ob.ant_q, n_iter=2, mu=1.0, nu=2.0)
    assert info.accepted == [False, False]
    assert info.mus == [2.0, 8.0] and info.nus == [4.0, 8.0]
    assert np.array_equal(J, J0)


def test_zero_start_fails_to_factor_every_step():
    # fresh start at J = 0: H = 0, so mu_0 = tau * max diag H = 0 and the floor is 0 too;
    # the zero matrix has no Cholesky factor, so each iteration is a failed factorisation
    # counted as a rejection (mu stays 0, nu doubles)
    ob, V, C, x0, r, A = _setup(0.3, 2)
    J0 = np.zeros((ob.N, 2, 2), dtype=np.complex128)
    J, info = lm.lm_solve(V, C, J0, ob.ant_p, ob.ant_q, n_iter=3)
    assert (info.n_notpd, info.n_reject, info.n_accept) == (3, 3, 0)
    assert info.mu_effs == [0.0, 0.0, 0.0] and info.mus == [0.0, 0.0, 0.0]
    assert info.nus == [4.0, 8.0, 16.0]
    assert np.array_equal(J, J0)
    fV = float(np.sum(np.abs(V) ** 2))
    assert abs(info.cost - fV) <= 1e-12 * fV                      # f at J = 0 is ||V||^2
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(np.zeros((8 * ob.N, 8 * ob.N)))


@pytest.mark.parametrize("mu_rel, floor_active", [(1e-12, True), (1e-2, False)])
def test_mu_floor(mu_rel, floor_active):
    # mu_eff = max(mu, mu_floor * max diag): the step taken is the one damped by mu_eff
    ob, V, C, x0, r, A = _setup(0.3, 3)
    md = float(np.max(np.sum(A * A, axis=0)))
    mu = mu_rel * md
    mu_eff = max(mu, 1e-6 * md)
    assert (mu_eff > mu) == floor_active
    d, f, f_new, rho = _gain_ratio(ob, V, C, x0, r, A, mu_eff)
    # called with the default floor: the reading is 1e-6 of max diag (the library's default)
    J1, info = lm.lm_solve(V, C, _x_to_J(x0), ob.ant_p, ob.ant_q, n_iter=1, mu=mu, nu=2.0)
    assert info.accepted == [True]
    assert abs(info.mu_effs[0] - mu_eff) <= 1e-12 * mu_eff
    assert np.max(np.abs(_J_to_x(J1) - (x0 + d))) <= 1e-8 * np.max(np.abs(d))
    # the update scales mu, not mu_eff
    expect = mu * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
    assert abs(info.mu - expect) <= 1e-9 * expect
