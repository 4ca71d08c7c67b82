"""torch.autograd.Function over the C ABI: nsteps fixed-dt SSPRK steps of a
block list (Porth et al. 2014, Sect. 2.3) whose backward is the hand-written
adjoint with checkpoint-and-recompute (amrvac_ssprk_adjoint).

Only marshalling happens here; forward and backward run in the native
library on the tensors' device.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import amrvac


class BlockSolver:
    """A context plus the block geometry (n, dx, xlo, nbr) of a block list."""

    def __init__(self, ndim: int, mhd: bool, gamma: float, n, dx, xlo, nbr):
        self.ctx = amrvac.Context(ndim, mhd, gamma)
        self.geom = (n, dx, xlo, nbr)

    def bind(self, states: Sequence[torch.Tensor]):
        self.ctx.set_blocks(list(states), *self.geom)

    def close(self):
        self.ctx.close()


class SSPRKSteps(torch.autograd.Function):
    """U_N = SSPRKSteps.apply(solver, scheme, dt, nsteps, ckpt_every, *U_0).

    U_0 / U_N: float64 device tensors in the padded block layout.  The
    gradient returned for each U_0 block has zero ghost layers (for periodic
    faces the ghost entries are not inputs of the scheme)."""

    @staticmethod
    def forward(ctx, solver: BlockSolver, scheme: int, dt: float, nsteps: int, ckpt_every: int,
                *u0: torch.Tensor):
        outs = [u.detach().clone().contiguous() for u in u0]
        solver.bind(outs)
        # t=0.0 waits for the steps and reads the device status, so a
        # non-physical forward state raises here rather than in backward
        solver.ctx.ssprk_step(scheme, nsteps, dt=dt, t=0.0)
        ctx.solver, ctx.scheme, ctx.dt, ctx.nsteps, ctx.ckpt = solver, scheme, dt, nsteps, ckpt_every
        ctx.save_for_backward(*u0)
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads: torch.Tensor):
        u0 = ctx.saved_tensors
        lam = [(g if g is not None else torch.zeros_like(u)).detach().clone().contiguous()
               for g, u in zip(grads, u0)]
        ctx.solver.bind([u.detach().contiguous() for u in u0])
        ctx.solver.ctx.ssprk_adjoint(ctx.scheme, ctx.dt, ctx.nsteps, ctx.ckpt, lam)
        return (None, None, None, None, None, *lam)
