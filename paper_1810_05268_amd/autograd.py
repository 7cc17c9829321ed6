"""torch.autograd.Function: interior velocity -> misfit, through the C ABI.

Forward: the interior velocity is extended into the absorbing layer
(``wv_pad_velocity``), then one checkpointed sweep (``wv_misfit_gradient``)
computes d_sim, the binary64 misfit of eq. (8) and the adjoint-state gradient
with respect to m = 1/c^2; ``wv_velocity_gradient`` maps it to the interior
velocity (dm/dc = -2/c^3, then the adjoint of the padding).  Backward scales that
gradient by the incoming gradient.  Checkpointing (and, with tol > 0, the codec)
is the memory strategy of the sweep.  Every step runs in libwv.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B
from .shot import DeviceShot


class WaveProblem:
    """Everything of one shot except the velocity: grid, time stepping, geometry,
    wavelet, observed data and the checkpoint settings."""

    def __init__(self, ndim, n, h, nbl, space_order, nt, dt, vmax, wavelet, src, rec, d_obs, mem_budget,
                 tol=0.0, ratio_hint=0.0, device="cuda"):
        self.ndim, self.n, self.nbl = ndim, tuple(n), nbl
        padded = tuple(reversed([n[a] + 2 * nbl for a in range(ndim)]))
        self.shot = DeviceShot(ndim, n, h, nbl, space_order, nt, dt, vmax, np.ones(padded, np.float32) * vmax,
                               wavelet, src, rec, device=device)
        self.d_obs = torch.as_tensor(np.ascontiguousarray(d_obs, dtype=np.float32), device=device) \
            if not isinstance(d_obs, torch.Tensor) else d_obs
        self.mem_budget, self.tol, self.ratio_hint = int(mem_budget), float(tol), float(ratio_hint)
        self.last_stats = None
        self.vel_padded = torch.empty(padded, dtype=torch.float32, device=device)


class WaveMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vel, problem: WaveProblem):
        v = vel.detach().to(torch.float32).contiguous()
        B.pad_velocity(problem.ndim, problem.n, problem.nbl, v, problem.vel_padded)
        problem.shot.set_velocity(problem.vel_padded)
        phi, gm, st = problem.shot.misfit_gradient(problem.d_obs, problem.mem_budget, problem.tol,
                                                   problem.ratio_hint)
        problem.last_stats = st
        if problem.tol > 0 and problem.ratio_hint <= 0 and all(x > 0 for x in st["profile"]):
            # plan later calls from the compressibility this one measured (they skip the
            # unhinted first attempt that stores every state)
            _, h = B.plan(problem.shot.nt, problem.shot.P, problem.mem_budget, st["profile"])
            problem.ratio_hint = h if h > 0 else 0.95 * st["ratio_planned"]
        gv = torch.empty(v.shape, dtype=torch.float64, device=v.device)
        B.velocity_gradient(problem.ndim, problem.n, problem.nbl, problem.vel_padded, gm, gv)
        ctx.save_for_backward(gv)
        ctx.vel_dtype = vel.dtype
        return torch.tensor(phi, dtype=torch.float64, device=vel.device)

    @staticmethod
    def backward(ctx, grad_out):
        (gv,) = ctx.saved_tensors
        return (grad_out * gv).to(ctx.vel_dtype), None


def wave_misfit(vel: torch.Tensor, problem: WaveProblem) -> torch.Tensor:
    return WaveMisfit.apply(vel, problem)
