"""MAP reconstruction of the initial conditions from an observed final
overdensity (section 7 of the paper, reconstruction from dark matter).

Every iteration is one library call (``pm_recon_step``): Gen-IC from the
current white noise, the KDK run with checkpoints, the chi^2 residual, the
adjoint of the run and the Adam update, all in the HIP library.  This module
only owns the buffers (noise, Adam moments, work space) and counts steps.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import torch

from .binding import PMContext, PMError


class Reconstruction:
    """Adam on loss(w) = sum ((delta_m(w) - data) / sigma)^2 + sum w^2.

    The paper's text uses learning rate 0.01 (its listing 0.1)."""

    def __init__(self, ctx: PMContext, a_list: Sequence[float], data: torch.Tensor, sigma: float,
                 noise0: Optional[torch.Tensor] = None, lr: float = 0.01, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8):
        n = ctx.workload.n_part
        self.ctx, self.a_list, self.data, self.sigma = ctx, list(a_list), data, float(sigma)
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        if noise0 is None:
            self.noise = torch.zeros((n, n, n), dtype=torch.float32, device=ctx.device)
        else:
            self.noise = noise0.detach().clone().contiguous()
        self.m = torch.zeros_like(self.noise)
        self.v = torch.zeros_like(self.noise)
        self.work = torch.empty(ctx.pm_recon_work_bytes(len(self.a_list)), dtype=torch.uint8, device=ctx.device)
        self.t = 0
        self.history: List[Tuple[float, float]] = []

    def step(self) -> Tuple[float, float]:
        """One iteration; returns (chi^2, prior) at the noise before the update."""
        self.t += 1
        out = self.ctx.pm_recon_step(self.a_list, self.data, self.sigma, self.noise, self.m, self.v, self.t,
                                     self.lr, self.beta1, self.beta2, self.eps, work=self.work)
        self.history.append(out)
        return out

    def run(self, n_iter: int) -> List[Tuple[float, float]]:
        if n_iter < 0:
            raise PMError("n_iter must be >= 0")
        return [self.step() for _ in range(n_iter)]
