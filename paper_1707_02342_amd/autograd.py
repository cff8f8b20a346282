"""torch.autograd.Function over the library's objective/adjoint entry points.

    J = -lambda log((1/K) sum_k exp(-S_k / lambda))

the Monte-Carlo free energy of one MPPI iteration's samples (Eq. FreeEnergy), as a
differentiable function of the nominal controls U ([T][2]) and the packed dynamics
network parameters (1412 floats).  Forward and backward both run in the library's
HIP kernels (the backward is the hand-written adjoint rollout with checkpoints);
this module only moves tensors across the C ABI.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mppi as M


class FreeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U: torch.Tensor, params: torch.Tensor, controller: "M.Controller", x0,
                it: int, ckpt_every: int = 10):
        controller.set_controls(U.detach().to("cpu", torch.float32).numpy())
        controller.set_dynamics(params.detach().to("cpu", torch.float32).numpy())
        J, _ = controller.objective(np.asarray(x0, np.float32), it, ckpt_every)
        ctx.controller = controller
        ctx.devices = (U.device, params.device)
        return torch.tensor(J, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        gU, gth = ctx.controller.objective_backward()
        g = float(gJ.detach().cpu())
        dU = torch.from_numpy(gU).to(ctx.devices[0]) * g
        dth = torch.from_numpy(gth).to(ctx.devices[1]) * g
        return dU, dth, None, None, None, None


def free_energy(U: torch.Tensor, params: torch.Tensor, controller: "M.Controller", x0, it: int = 0,
                ckpt_every: int = 10) -> torch.Tensor:
    return FreeEnergy.apply(U, params, controller, x0, it, ckpt_every)
