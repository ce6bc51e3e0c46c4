"""Gradient of the calibration cost with respect to every cluster's Jones (FP64).

Test infrastructure only (see ``oracle/__init__``).

f(x) = ||V - sum_k M_k(x_k)||^2 with M_k = J_{p,k} C_k J_{q,k}^H (measurement equation;
paper Section 2: one solution per cluster).  In the real-pair parameter view x_k (see
``normal_eq``), df/dx_k = -2 A_k^T r with r the full residual and A_k = dM_k/dx_k, i.e.
-2 times the normal-equation right-hand side of cluster k evaluated on Y_k = r + M_k.
Written here through the brute-force Jacobian blocks of ``normal_eq``.
"""
from __future__ import annotations

import numpy as np

from .normal_eq import normal_equations
from .rime import model_cluster, residual, cost


def cost_and_gradient(Vis, C, J, ant_p, ant_q):
    """(f, grad) with grad[k] = df/dx_k as [N, 8] (real pairs of the 2x2 entries)."""
    R = residual(Vis, C, J, ant_p, ant_q)
    f = cost(R)
    K, N = J.shape[0], J.shape[1]
    grad = np.empty((K, N, 8))
    for k in range(K):
        Yk = R + model_cluster(C[k], J[k], ant_p, ant_q)
        _, g, _ = normal_equations(Yk, C[k], J[k], ant_p, ant_q)
        grad[k] = -2.0 * g.reshape(N, 8)
    return f, grad
