"""Differentiable calibration cost for torch, backed by the library's adjoint kernel.

``CalibrationCost.apply(jones, problem)`` returns f = ||V - sum_k J_k C_k J_k^H||^2 as a
0-d float64 tensor; its backward multiplies the gradient that ``ddc_cost_gradient`` (the
hand-written adjoint kernel) produced in the same pass.  ``jones`` is the float64
[K, N, 8] real-pair view used by the C ABI, so ``jones.grad`` is df/dx directly.

``lbfgs_calibrate`` drives ``torch.optim.LBFGS`` with it: the gradient-based alternative to
the Levenberg-Marquardt solve.  The optimiser's own vector arithmetic runs as torch ops on
the device; every cost and gradient evaluation runs in the library's HIP kernels.
"""
from __future__ import annotations

import dataclasses
from typing import List

import torch

from . import ddcal as dd


@dataclasses.dataclass
class Problem:
    ctx: "dd.Context"
    obs: "dd.DeviceObs"
    K: int
    vis: torch.Tensor        # [8, T, F, B]
    coh: torch.Tensor        # [K, 8, T, F, B]
    precision: int = dd.MIXED


class CalibrationCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, jones: torch.Tensor, problem: Problem):
        j = jones.detach().contiguous()
        if jones.requires_grad:
            cost, grad = problem.ctx.cost_gradient(problem.obs, problem.K, problem.vis, problem.coh,
                                                   j, problem.precision)
            ctx.save_for_backward(grad)
        else:
            cost = problem.ctx.residual(problem.obs, problem.K, problem.vis, problem.coh, j,
                                        problem.precision, None)
        return torch.tensor(cost, dtype=torch.float64, device=jones.device)

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return gout * grad, None


def calibration_cost(jones: torch.Tensor, problem: Problem) -> torch.Tensor:
    return CalibrationCost.apply(jones, problem)


def lbfgs_calibrate(problem: Problem, jones0: torch.Tensor, n_iter: int = 200,
                    history: int = 20, lr: float = 1.0):
    """Minimise the cost over all clusters' Jones with L-BFGS (strong-Wolfe line search).

    Returns (jones, costs) with costs the cost after each outer iteration.
    """
    x = jones0.detach().clone().requires_grad_(True)
    opt = torch.optim.LBFGS([x], lr=lr, max_iter=1, history_size=history,
                            line_search_fn="strong_wolfe", tolerance_grad=0.0,
                            tolerance_change=0.0)
    costs: List[float] = []

    def closure():
        opt.zero_grad()
        f = calibration_cost(x, problem)
        f.backward()
        return f

    for _ in range(n_iter):
        f = opt.step(closure)
        costs.append(float(f))
    return x.detach(), costs
