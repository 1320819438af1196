"""torch.autograd.Function around the PM forward run and its hand-written adjoint.

Forward: white noise -> Gen-IC (LPT) -> KDK run -> final overdensity, with
the particle state checkpointed at every scale factor.  Backward: the
library's reverse sweep (pm_run_adjoint), which recomputes the force meshes
from the checkpointed positions.  No autodiff of the kernels is involved.
"""
from __future__ import annotations

from typing import Sequence

import torch

from .binding import PMContext


class _PMSimulation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, noise: torch.Tensor, pm: PMContext, a_list: Sequence[float]):
        noise = noise.detach().contiguous()
        pos, mom = pm.pm_init_lpt(0, a_list[0], noise=noise)
        n = pm.workload.n_mesh
        ckpt = torch.empty((len(a_list), 2, pm.np3, 3), dtype=torch.float32, device=noise.device)
        delta = torch.empty((n, n, n), dtype=torch.float32, device=noise.device)
        pm.pm_run(a_list, pos, mom, ckpt=ckpt, delta_final=delta)
        ctx.save_for_backward(noise, ckpt)
        ctx.pm = pm
        ctx.a_list = tuple(a_list)
        return delta

    @staticmethod
    def backward(ctx, grad_delta: torch.Tensor):
        noise, ckpt = ctx.saved_tensors
        _, _, gn = ctx.pm.pm_run_adjoint(ctx.a_list, ckpt, noise=noise, grad_delta=grad_delta.contiguous())
        return gn, None, None


def simulate(noise: torch.Tensor, pm: PMContext, a_list: Sequence[float]) -> torch.Tensor:
    """Final overdensity of a PM run from white noise; differentiable in noise."""
    return _PMSimulation.apply(noise, pm, a_list)
