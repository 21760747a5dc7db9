"""torch.autograd binding of the one-centre propagation and its adjoint.

``propagate_probabilities(b, a, c, ...)`` returns the final probabilities
P[j, i] = |X_j,i|^2 of Algorithm 1 for paths with impact parameters b and the
screened target potential -(1 + a e^{-c r})/r; its backward pass calls
``wpccc_adjoint`` (reverse mode through every RK4 step, checkpointed states)
for dL/db per path and dL/da, dL/dc summed over the paths.  Argument
marshalling only: all arithmetic runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (Basis, wpccc_adjoint, wpccc_plan_create, wpccc_plan_path_info, wpccc_plan_status,
               wpccc_propagate)


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, a, c, basis, v, zgrid, Zp, checkpoint_every):
        bh = b.detach().to("cpu", torch.float64).numpy()
        plan = wpccc_plan_create(basis, bh, v, Zp=Zp, model_a=float(a), model_c=float(c),
                                 checkpoint_every=checkpoint_every)
        N = wpccc_plan_path_info(plan, 0)[0]
        X0 = torch.zeros((plan.n_traj, plan.n_pad), dtype=torch.complex128, device="cuda")
        X0[:, 0] = 1.0
        X = X0.clone()
        wpccc_propagate(plan, zgrid, X)
        wpccc_plan_status(plan)
        ctx.plan, ctx.zgrid, ctx.N = plan, np.asarray(zgrid, dtype=np.float64), N
        ctx.save_for_backward(X0, X)
        ctx.b_device = b.device
        return (X.abs() ** 2)[:, :N].to(torch.float64)

    @staticmethod
    def backward(ctx, gP):
        X0, X = ctx.saved_tensors
        plan, N = ctx.plan, ctx.N
        gX = torch.zeros_like(X)
        gX[:, :N] = gP.to(X.device, torch.float64) * X[:, :N]   # dL/d conj(X) = (dL/dP) X
        grad = torch.empty((plan.n_traj, 3), dtype=torch.float64, device="cuda")
        wpccc_adjoint(plan, ctx.zgrid, X0, gX, grad)
        gb = grad[:, 2].to(ctx.b_device)
        ga = grad[:, 0].sum().to(ctx.b_device)
        gc = grad[:, 1].sum().to(ctx.b_device)
        return gb, ga, gc, None, None, None, None, None


def propagate_probabilities(b: torch.Tensor, a: torch.Tensor, c: torch.Tensor, basis: Basis, v,
                            zgrid, Zp: float = 1.0, checkpoint_every: int = 0) -> torch.Tensor:
    """Final probabilities [n_paths, N] as a differentiable function of b, a and c."""
    return _Propagate.apply(b, a, c, basis, v, zgrid, Zp, checkpoint_every)
