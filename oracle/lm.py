"""Levenberg-Marquardt for one cluster and the SAGE sweep over clusters, in FP64.

Test infrastructure only (see ``oracle/__init__``).

The paper states the problem (Section 2: one calibration solution per cluster; Section 3:
N(N-1)/2 baselines) but not the solver.  The solver here is Levenberg-Marquardt with
Levenberg damping mu*I as in Madsen, Nielsen & Tingleff, "Methods for non-linear least
squares problems" (2004), Algorithm 3.16, applied to f(x) = ||Y - M(x)||^2 (no factor 1/2):

    H = A^T A, g = A^T r                        (normal equations at x)
    mu_eff = max(mu, mu_floor * max diag H)     (floor against the gauge null space)
    (H + mu_eff I) d = g                        (Cholesky, then two triangular solves)
    rho = (f(x) - f(x + d)) / (d . (mu_eff d + g))
    rho > 0: x <- x + d, mu <- mu * max(1/3, 1 - (2 rho - 1)^3), nu <- 2
    else:    mu <- mu * nu, nu <- 2 nu

The denominator is the exact decrease of the linear model ||r - A d||^2, since
(H + mu_eff I) d = g.  Readings (the paper is silent on all of them): identity start,
mu_0 = tau * max diag H with tau = 1e-3, nu_0 = 2, strict rho > 0, a rejected step counts
as an iteration, a failed factorisation or a non-positive or non-finite denominator counts
as a rejection, and H is rebuilt only after an accepted step (it is unchanged otherwise).

SAGE (space-alternating generalised EM; the scheme SAGECal is named after) visits the
clusters in index order each sweep: Y_k = R + J_k C_k J_k^H, LM on Y_k, R = Y_k - J_k' C_k J_k'^H.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
from scipy.linalg import solve_triangular

from .normal_eq import normal_equations, pack_jones, unpack_jones
from .rime import model_cluster, cost


@dataclasses.dataclass
class LMInfo:
    cost0: float = 0.0
    cost: float = 0.0
    n_accept: int = 0
    n_reject: int = 0
    n_notpd: int = 0
    mu: float = 0.0
    nu: float = 2.0
    costs: List[float] = dataclasses.field(default_factory=list)   # f(x) after each iteration
    accepted: List[bool] = dataclasses.field(default_factory=list)
    mu_effs: List[float] = dataclasses.field(default_factory=list)  # damping used in each iteration
    mus: List[float] = dataclasses.field(default_factory=list)      # mu after each iteration
    nus: List[float] = dataclasses.field(default_factory=list)      # nu after each iteration
    trial_costs: List[float] = dataclasses.field(default_factory=list)  # f(x + d) (nan: no step)


def damped_solve(H, g, mu_eff):
    """d with (H + mu_eff I) d = g by Cholesky; None if the factorisation fails."""
    A = H + mu_eff * np.eye(H.shape[0])
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return None
    y = solve_triangular(L, g, lower=True)
    return solve_triangular(L.T, y, lower=False)


def lm_solve(Y, C, J0, ant_p, ant_q, n_iter, tau=1e-3, mu_floor=1e-6,
             mu: Optional[float] = None, nu: float = 2.0):
    """Run ``n_iter`` LM iterations for one cluster from Jones J0 ([N, 2, 2]).

    Passing back ``mu`` and ``nu`` from a previous ``LMInfo`` resumes the iteration.
    Returns (J, LMInfo).
    """
    J = np.array(J0, dtype=np.complex128)
    x = pack_jones(J)
    H, g, f = normal_equations(Y, C, J, ant_p, ant_q)
    info = LMInfo(cost0=f)
    if mu is None:
        mu = tau * float(np.max(np.diag(H)))
        nu = 2.0
    for _ in range(n_iter):
        mu_eff = max(mu, mu_floor * float(np.max(np.diag(H))))
        d = damped_solve(H, g, mu_eff)
        accepted = False
        f_new = float("nan")
        if d is None:
            info.n_notpd += 1
        else:
            x_new = x + d
            f_new = cost(Y - model_cluster(C, unpack_jones(x_new), ant_p, ant_q))
            denom = float(d @ (mu_eff * d + g))
            if denom > 0.0 and np.isfinite(denom) and np.isfinite(f_new):
                rho = (f - f_new) / denom
                if rho > 0.0:
                    accepted = True
                    x = x_new
                    mu = mu * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
                    nu = 2.0
        if accepted:
            info.n_accept += 1
            H, g, f = normal_equations(Y, C, unpack_jones(x), ant_p, ant_q)
        else:
            info.n_reject += 1
            mu = mu * nu
            nu = 2.0 * nu
        info.costs.append(f)
        info.accepted.append(accepted)
        info.mu_effs.append(mu_eff)
        info.mus.append(mu)
        info.nus.append(nu)
        info.trial_costs.append(f_new)
    info.cost = f
    info.mu, info.nu = mu, nu
    return unpack_jones(x), info


def calibrate(Vis, C, J0, ant_p, ant_q, n_sweeps, n_lm, tau=1e-3, mu_floor=1e-6,
              track_total_cost=False):
    """SAGE sweep: for each sweep, for each cluster in order, LM on Y_k = R + model_k.

    Vis: [T, F, B, 2, 2]; C: [K, T, F, B, 2, 2]; J0: [K, N, 2, 2].
    Returns (J, R, infos, totals) with infos[e][k] the LMInfo of cluster k in sweep e and
    totals the total cost ||R||^2 after every cluster update (if requested).
    """
    K = C.shape[0]
    J = np.array(J0, dtype=np.complex128)
    R = np.array(Vis, dtype=np.complex128)
    for k in range(K):
        R -= model_cluster(C[k], J[k], ant_p, ant_q)
    infos, totals = [], []
    if track_total_cost:
        totals.append(cost(R))
    for _ in range(n_sweeps):
        row = []
        for k in range(K):
            Y = R + model_cluster(C[k], J[k], ant_p, ant_q)
            J[k], info = lm_solve(Y, C[k], J[k], ant_p, ant_q, n_lm, tau=tau, mu_floor=mu_floor)
            R = Y - model_cluster(C[k], J[k], ant_p, ant_q)
            row.append(info)
            if track_total_cost:
                totals.append(cost(R))
        infos.append(row)
    return J, R, infos, totals
