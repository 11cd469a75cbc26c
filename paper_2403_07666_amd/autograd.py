"""torch.autograd.Function over the coil run and its hand-written adjoint.

    obj = CoilObjective.apply(c_wire, ramp, coil, nsteps)   # tensor [Q, T_peak]
    obj[0].backward()   # -> c_wire.grad, ramp.grad from coil_adjoint

Forward sets the parameters on the handle, resets it and runs nsteps steps
(coil_run); backward calls coil_adjoint with the incoming gradient of
(Q, T_peak) as the objective weights (checkpoints every 50 steps).  Parameters
and results are float64 CPU tensors; the state lives on the GPU.
"""
from __future__ import annotations

import numpy as np
import torch


class CoilObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c_wire: torch.Tensor, ramp: torch.Tensor, coil, nsteps: int,
                ckpt_every: int = 50):
        cw = c_wire.detach().cpu().double().numpy()
        rp = ramp.detach().cpu().double().numpy()
        coil.set_params(cw, rp)
        Q, Tp = coil.objectives(nsteps)
        ctx.coil = coil
        ctx.nsteps = int(nsteps)
        ctx.ckpt = int(ckpt_every)
        ctx.params = (cw, rp)
        return torch.tensor([Q, Tp], dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = grad_out.detach().cpu().double().numpy()
        coil = ctx.coil
        cw, rp = ctx.params
        coil.set_params(cw, rp)
        gcw, gr, _ = coil.adjoint(ctx.nsteps, wQ=float(g[0]), wT=float(g[1]), ckpt_every=ctx.ckpt)
        return (torch.from_numpy(np.asarray(gcw)), torch.from_numpy(np.asarray(gr)), None, None, None)
