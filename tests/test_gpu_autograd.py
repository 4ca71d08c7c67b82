"""SSPRKSteps (torch.autograd.Function) gives the C-ABI adjoint's gradient
and matches the oracle's JVP in a random direction."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1407_2052_amd import amrvac as A  # noqa: E402
from paper_1407_2052_amd.autograd import BlockSolver, SSPRKSteps  # noqa: E402


def test_density_misfit_gradient_through_autograd():
    print("[autograd] 2D hydro 64^2 density misfit", flush=True)
    bs = inputs.hydro_random_2d(64, 16, seed=4)
    target = [t[:, :16, :16] for t in inputs.hydro_target_density(64, 16, seed=40)]
    _, cm = oracle.rhs(bs)
    dt = 0.4 / sum(cm[d] / bs.dx[0, d] for d in range(2))
    nsteps, ckpt = 12, 5
    solver = BlockSolver(bs.ndim, bs.mhd, bs.gamma, bs.n, bs.dx, bs.xlo, bs.nbr)
    u0 = [torch.from_numpy(u.copy()).cuda().requires_grad_(True) for u in bs.u]
    uN = SSPRKSteps.apply(solver, A.SSPRK54, dt, nsteps, ckpt, *u0)
    tgt = [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in target]
    loss = sum(0.5 * ((u[0, :, 3:-3, 3:-3] - t) ** 2).sum() for u, t in zip(uN, tgt))
    loss.backward()
    grads = [u.grad.cpu().numpy() for u in u0]
    # same as the C ABI called directly
    lam = []
    for b, u in enumerate(uN):
        x = torch.zeros_like(u)
        x[0, :, 3:-3, 3:-3] = u[0, :, 3:-3, 3:-3].detach() - tgt[b]
        lam.append(x.contiguous())
    ctx, flat, views = A.context_for(bs)
    ctx.ssprk_adjoint(A.SSPRK54, dt, nsteps, ckpt, lam)
    for g, l in zip(grads, lam):
        assert np.array_equal(g, l.cpu().numpy())
    ctx.close()
    # directional derivative against the oracle's forward mode (density only)
    tang = inputs.random_tangent(bs, 17, vars_=[0])
    out, du = oracle.run_jvp(bs, tang, oracle.SSPRK54, nsteps, dt)
    dirder = math.fsum(float(((out.interior(b)[0] - target[b]) * bs.interior(b, du[b])[0]).sum())
                       for b in range(bs.nb))
    got = math.fsum(float((bs.interior(b, grads[b]) * bs.interior(b, tang[b])).sum()) for b in range(bs.nb))
    assert abs(got - dirder) <= 1e-10 * abs(dirder), (got, dirder)
    solver.close()
