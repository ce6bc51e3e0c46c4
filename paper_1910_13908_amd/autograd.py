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


def jacobi_scaling(problem: Problem, jones0: torch.Tensor, floor: float = 1e-12) -> torch.Tensor:
    """Per-parameter scale diag(A_k^T A_k)^{-1/2} of every cluster's normal equations at jones0
    (built by the library from the full data, as in the first LM iteration), shape [K, N, 8]."""
    K = problem.K
    out = torch.empty_like(jones0)
    for k in range(K):
        JtJ, _, _ = problem.ctx.build_normal_eq(problem.obs, problem.vis, problem.coh[k].contiguous(),
                                                jones0[k].contiguous(), problem.precision)
        d = torch.diagonal(JtJ).to(torch.float64).reshape(out.shape[1], 8)
        out[k] = torch.rsqrt(torch.clamp(d, min=floor * float(d.max())))
    return out


def lbfgs_calibrate(problem: Problem, jones0: torch.Tensor, n_iter: int = 200,
                    history: int = 20, lr: float = 1.0, scaling: torch.Tensor = None):
    """Minimise the cost over all clusters' Jones with L-BFGS (strong-Wolfe line search).

    With ``scaling`` (e.g. ``jacobi_scaling``) the optimiser works on z, x = jones0 + scaling * z:
    a diagonal change of variables (preconditioner), the cost and its gradient unchanged.
    Returns (jones, costs) with costs the cost after each outer iteration.
    """
    x0 = jones0.detach().clone()
    s = scaling.detach() if scaling is not None else None
    z = torch.zeros_like(x0).requires_grad_(True) if s is not None else x0.clone().requires_grad_(True)
    opt = torch.optim.LBFGS([z], lr=lr, max_iter=1, history_size=history,
                            line_search_fn="strong_wolfe", tolerance_grad=0.0,
                            tolerance_change=0.0)
    costs: List[float] = []

    def point():
        return x0 + s * z if s is not None else z

    def closure():
        opt.zero_grad()
        f = calibration_cost(point(), problem)
        f.backward()
        return f

    for _ in range(n_iter):
        f = opt.step(closure)
        costs.append(float(f.detach()))
    return point().detach(), costs
