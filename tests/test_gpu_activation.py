"""GPU dynamic grid activation (the paper's appendix "Dynamic grid
activation") against the oracle's masked integration: only active blocks are
advanced, passive blocks keep their state and feed their neighbours' halos,
c_max and the time step come from the active blocks.

Bar: states to 1e-11 relative L1 per variable after the steps, passive
interiors bitwise unchanged, execution forms bitwise equal."""
import sys

import numpy as np
import pytest

import oracle
from helpers import rel_l1, strip_blocks
from paper_1407_2052_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1407_2052_amd import amrvac as A  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "ot2d": lambda: inputs.orszag_tang_2d(64, 16),
    "uneven3d": lambda: inputs.uneven_3d(nblocks=14, seed=3, N=64),
    "ragged2d_hd": lambda: strip_blocks(2, False, [13, 19, 7, 9], ny=10, seed=1, gamma=1.4),
}


def mask_for(bs, seed, frac=0.35, first_passive=False):
    rng = np.random.default_rng(seed)
    want = rng.random(bs.nb) >= frac
    if first_passive:
        want[0] = False
    want[1] = True
    return want.astype(np.uint8)


def gpu_masked_run(bs, flags, scheme, nsteps, exec=A.EXEC_BATCHED, dt=None):
    ctx, flat, views = A.context_for(bs, exec)
    ctx.set_active(flags)
    t = ctx.ssprk_step(scheme, nsteps, cfl=0.4, dt=dt, t=0.0)
    out = bs.copy()
    out.u = [v.cpu().numpy() for v in views]
    ctx.close()
    return out, t


def oracle_masked_run(bs, flags, scheme, nsteps, dt=None):
    oracle.set_active(flags)
    try:
        return oracle.run(bs, scheme, nsteps, cfl=0.4, dt=dt)
    finally:
        oracle.set_active(None)


@pytest.mark.parametrize("case,scheme,nsteps", [("ot2d", oracle.SSPRK54, 30), ("uneven3d", oracle.SSPRK54, 10),
                                                ("ragged2d_hd", oracle.RK3, 30)])
def test_masked_steps_match_oracle(case, scheme, nsteps):
    say(f"[active] {case}")
    bs = CASES[case]()
    flags = mask_for(bs, 5)
    out_o, dts = oracle_masked_run(bs, flags, scheme, nsteps)
    out_g, t = gpu_masked_run(bs, flags, scheme, nsteps)
    assert abs(t - dts.sum()) <= 1e-12 * dts.sum()
    for v in range(bs.nvar):
        num, den = rel_l1(out_g.u, out_o.u, bs, v)
        assert (num == 0.0) if den == 0.0 else num / den <= 1e-11, (v, num, den)
    for b in range(bs.nb):
        if not flags[b]:
            assert np.array_equal(out_g.interior(b), bs.interior(b)), b


def test_masked_rhs_matches_oracle_and_leaves_passive_arrays_alone():
    bs = CASES["ot2d"]()
    flags = mask_for(bs, 6)
    oracle.set_active(flags)
    try:
        Lo, cmo = oracle.rhs(bs)
    finally:
        oracle.set_active(None)
    ctx, flat, views = A.context_for(bs)
    ctx.set_active(flags)
    out = [torch.full((bs.nvar,) + tuple(int(x) for x in bs.n[b][::-1]), 7.25, dtype=torch.float64,
                      device="cuda") for b in range(bs.nb)]
    out_list, cm = ctx.fd_rhs(out)
    res = [o.cpu().numpy() for o in out_list]
    ctx.close()
    np.testing.assert_allclose(cm, cmo, rtol=1e-14)
    umax = max(float(np.abs(bs.interior(b)).max()) for b in range(bs.nb))
    scale = max(sum(cmo[d] * umax / bs.dx[b, d] for d in range(bs.ndim)) for b in range(bs.nb))
    for b in range(bs.nb):
        if flags[b]:
            assert np.abs(res[b].reshape(bs.interior(b).shape) - bs.interior(b, Lo[b])).max() <= 1e-14 * scale
        else:
            assert np.all(res[b] == 7.25)


@pytest.mark.parametrize("first_passive", [False, True])
def test_masked_per_block_launch_equals_batched(first_passive):
    bs = CASES["uneven3d"]()
    flags = mask_for(bs, 7, first_passive=first_passive)
    a, ta = gpu_masked_run(bs, flags, oracle.SSPRK54, 4, exec=A.EXEC_PER_BLOCK)
    b, tb = gpu_masked_run(bs, flags, oracle.SSPRK54, 4, exec=A.EXEC_BATCHED)
    assert ta == tb
    for x, y in zip(a.u, b.u):
        assert np.array_equal(x, y)


def test_all_active_is_the_plain_run():
    bs = CASES["ot2d"]()
    ctx, flat, views = A.context_for(bs)
    ctx.set_active(np.zeros(bs.nb, np.uint8) + 1)
    ctx.set_active(None)
    t1 = ctx.ssprk_step(oracle.SSPRK54, 5, t=0.0)
    a = [v.cpu().numpy() for v in views]
    ctx.close()
    ctx, flat, views = A.context_for(bs)
    t2 = ctx.ssprk_step(oracle.SSPRK54, 5, t=0.0)
    b = [v.cpu().numpy() for v in views]
    ctx.close()
    assert t1 == t2
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_passive_blocks_are_rejected_where_unsupported():
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(2, [64, 64], [16, 16])
    bs = inputs.hydro_random_2d(64, 16, seed=4)
    ctx, flat, views = A.context_for(bs)
    flags = np.ones(bs.nb, np.uint8)
    flags[3] = 0
    ctx.set_active(flags)
    lam = [torch.zeros_like(v) for v in views]
    with pytest.raises(A.AmrvacError) as ei:
        ctx.ssprk_adjoint(oracle.SSPRK54, 1e-3, 1, 1, lam)
    assert ei.value.status == A.ERR_UNSUPPORTED
    with pytest.raises(A.AmrvacError) as ei:
        ctx.autotune(oracle.SSPRK54, 1)
    assert ei.value.status == A.ERR_UNSUPPORTED
    with pytest.raises(A.AmrvacError) as ei:
        ctx.set_active(np.zeros(bs.nb, np.uint8))
    assert ei.value.status == A.ERR_INVALID
    ctx.close()


@pytest.mark.parametrize("physics", ["glm", "hall_lim03"])
def test_masked_steps_with_glm_and_hall(physics):
    # passive blocks keep psi (no decay) and still supply the current their
    # active neighbours read as halo in Hall MHD
    say(f"[active] {physics}")
    base = inputs.orszag_tang_2d(64, 16)
    bs = inputs.as_glm(base, psi=0.01) if physics == "glm" else base
    flags = mask_for(bs, 7)
    recon, eta, scheme = (A.MP5, 0.0, oracle.SSPRK54) if physics == "glm" else (A.LIM03, 0.02, oracle.RK3)
    oracle.set_active(flags)
    oracle.set_recon(recon)
    oracle.set_hall(eta)
    try:
        out_o, dts = oracle.run(bs, scheme, 12, cfl=0.4)
    finally:
        oracle.set_active(None)
        oracle.set_recon(oracle.MP5)
        oracle.set_hall(0.0)
    ctx, flat, views = A.context_for(bs, recon=recon, eta_h=eta)
    ctx.set_active(flags)
    t = ctx.ssprk_step(scheme, 12, cfl=0.4, t=0.0)
    out_g = bs.copy()
    out_g.u = [v.cpu().numpy() for v in views]
    ctx.close()
    assert abs(t - dts.sum()) <= 1e-12 * dts.sum()
    dens = [rel_l1(out_o.u, out_o.u, bs, v)[1] for v in range(bs.nvar)]
    for v in range(bs.nvar):
        num, den = rel_l1(out_g.u, out_o.u, bs, v)
        assert num <= 1e-11 * max(den, 1e-3 * sum(dens)), (v, num, den)
    for b in range(bs.nb):
        if not flags[b]:
            assert np.array_equal(out_g.interior(b), bs.interior(b)), b
