"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.

Bar: right-hand sides element by element to 1e-14 of the size of the split
flux terms they difference (sum_d c_max,d max|U| / dx_d: L is a difference
of such terms, so rounding differences scale with them, not with |L|);
states after many steps to 1e-11 relative L1 per conserved variable
(variables the oracle keeps exactly zero must stay exactly zero); bitwise
equality between execution forms, block decompositions and repeated runs.
"""
import math
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

RTOL_STATE = 1e-11
RTOL_RHS = 1e-14


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_blocks(views):
    return [v.detach().cpu().numpy() for v in views]


def gpu_rhs(bs, exec=A.EXEC_BATCHED):
    ctx, flat, views = A.context_for(bs, exec)
    out, cm = ctx.fd_rhs()
    res = [o.cpu().numpy() for o in out]
    ctx.close()
    return res, cm


def gpu_run(bs, scheme, nsteps, cfl=0.4, dt=None, exec=A.EXEC_BATCHED):
    ctx, flat, views = A.context_for(bs, exec)
    t = ctx.ssprk_step(scheme, nsteps, cfl=cfl, dt=dt, t=0.0)
    out = bs.copy()
    out.u = host_blocks(views)
    ctx.close()
    return out, t


# ---------------------------------------------------------------- cases
def uneven_small(seed=3):
    # C3-like: mixed 32^3/16^3/8^3 blocks with fixed ghosts (1:2:4 by count)
    return inputs.uneven_3d(nblocks=14, seed=seed, N=64)


CASES = {
    "dwave1d": lambda: inputs.density_wave_1d(512),
    "dwave1d_8blk": lambda: inputs.density_wave_1d(512, nblocks=8),
    "sod1d_fixed": lambda: inputs.sod(128),
    "briowu1d_fixed": lambda: inputs.brio_wu(128),
    "ot2d": lambda: inputs.orszag_tang_2d(64, 16),
    "hydro2d": lambda: inputs.hydro_random_2d(64, 16, seed=4),
    "ragged2d_hd": lambda: strip_blocks(2, False, [13, 19, 7], ny=10, seed=1, gamma=1.4),
    "ragged2d_mhd": lambda: strip_blocks(2, True, [13, 19, 7], ny=21, seed=2),
    "ragged3d_mhd": lambda: strip_blocks(3, True, [9, 12], ny=7, nz=5, seed=3),
    "ragged3d_hd": lambda: strip_blocks(3, False, [10, 6], ny=9, nz=11, seed=4, gamma=1.4),
    "mhd3d": lambda: inputs.mhd_turbulence_3d(N=32, block=16, seed=5),
    "uneven3d": uneven_small,
    # the smallest blocks allowed (3 cells: a halo is a neighbour's whole
    # interior, or the block's own interior through the periodic wrap)
    "min3_1d_mhd": lambda: strip_blocks(1, True, [3, 5, 3, 3, 8, 3], seed=6),
    "min3_3d_mhd": lambda: strip_blocks(3, True, [3, 4, 3], ny=3, nz=3, seed=7),
    # one large block, periodic onto itself
    "big2d_single": lambda: big_single_block(),
}


def big_single_block(N=512):
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(2, [N, N], [N, N])
    from helpers import smooth_fields
    return inputs.sample_blocks(2, True, 5 / 3, n, dx, xlo, nbr, smooth_fields(2, True, 8, amp=0.08))


def rhs_scale(bs, cmax):
    umax = max(float(np.abs(bs.interior(b)).max()) for b in range(bs.nb))
    return max(sum(cmax[d] * umax / bs.dx[b, d] for d in range(bs.ndim)) for b in range(bs.nb))


def compare_rhs(bs, Lg, Lo, cmax):
    scale = rhs_scale(bs, cmax)
    worst = 0.0
    for b in range(bs.nb):
        g = Lg[b].reshape(bs.interior(b).shape)
        o = bs.interior(b, Lo[b])
        worst = max(worst, float(np.abs(g - o).max()))
    assert worst <= RTOL_RHS * max(scale, 1e-300), (worst, scale)
    return worst / scale


@pytest.mark.parametrize("case", sorted(CASES))
def test_rhs_matches_oracle(case):
    say(f"[rhs] {case}")
    bs = CASES[case]()
    Lo, cmo = oracle.rhs(bs)
    Lg, cmg = gpu_rhs(bs)
    np.testing.assert_allclose(cmg, cmo, rtol=1e-14, atol=0)
    compare_rhs(bs, Lg, Lo, cmo)


STEP_CASES = [
    ("dwave1d", oracle.RK3, 200),
    ("dwave1d", oracle.SSPRK54, 100),
    ("dwave1d_8blk", oracle.SSPRK43, 100),
    ("sod1d_fixed", oracle.SSPRK54, 100),
    ("briowu1d_fixed", oracle.SSPRK54, 60),
    ("ot2d", oracle.SSPRK54, 100),
    ("hydro2d", oracle.SSPRK54, 100),
    ("hydro2d", oracle.RK3, 100),
    ("ragged2d_hd", oracle.SSPRK54, 100),
    ("ragged2d_mhd", oracle.SSPRK43, 60),
    ("ragged3d_mhd", oracle.SSPRK54, 100),
    ("ragged3d_hd", oracle.RK3, 100),
    ("mhd3d", oracle.SSPRK54, 100),
    ("uneven3d", oracle.SSPRK54, 100),
    ("min3_1d_mhd", oracle.SSPRK54, 50),
    ("min3_3d_mhd", oracle.RK3, 10),
    ("big2d_single", oracle.SSPRK54, 2),
]


def assert_state_parity(bs, out_g, out_o, tol=RTOL_STATE):
    for v in range(bs.nvar):
        num, den = rel_l1(out_g.u, out_o.u, bs, v)
        if den == 0.0:
            assert num == 0.0, f"var {v} must stay exactly zero"
        else:
            assert num / den <= tol, (v, num / den)


@pytest.mark.parametrize("case,scheme,nsteps", STEP_CASES,
                         ids=[f"{c}-s{s}-n{n}" for c, s, n in STEP_CASES])
def test_steps_match_oracle(case, scheme, nsteps):
    say(f"[steps] {case} scheme={scheme} n={nsteps}")
    bs = CASES[case]()
    out_o, dts = oracle.run(bs, scheme, nsteps, cfl=0.4)
    out_g, t = gpu_run(bs, scheme, nsteps, cfl=0.4)
    assert abs(t - dts.sum()) <= 1e-12 * dts.sum()
    assert_state_parity(bs, out_g, out_o)


def test_fixed_dt_steps_match_oracle():
    bs = CASES["ot2d"]()
    say("[steps] ot2d fixed dt")
    out_o, _ = oracle.run(bs, oracle.SSPRK54, 50, dt=1e-4)
    out_g, t = gpu_run(bs, oracle.SSPRK54, 50, dt=1e-4)
    assert abs(t - 50e-4) < 1e-15
    assert_state_parity(bs, out_g, out_o)


@pytest.mark.parametrize("case", ["ot2d", "uneven3d", "ragged3d_mhd", "dwave1d_8blk"])
def test_execution_forms_are_bitwise_identical(case):
    say(f"[exec] {case}")
    bs = CASES[case]()
    a, ta = gpu_run(bs, oracle.SSPRK54, 5, exec=A.EXEC_PER_BLOCK)
    b, tb = gpu_run(bs, oracle.SSPRK54, 5, exec=A.EXEC_BATCHED)
    c, tc = gpu_run(bs, oracle.SSPRK54, 5, exec=A.EXEC_BATCHED_SINGLE)
    assert ta == tb == tc
    for x, y, z in zip(a.u, b.u, c.u):
        assert np.array_equal(x, y) and np.array_equal(x, z)


@pytest.mark.parametrize("case", ["ot2d", "uneven3d"])
def test_multi_step_graph_replays_equal_eager_launches(case):
    """Calls long enough to replay the multi-step graph (8 steps per graph,
    the remainder on the one-step graph), several in a row with eager work
    and synchronisations between them, against the per-block form (kernels
    launched one by one, no graph) on the same call pattern: bitwise equal
    after every call."""
    import torch
    say(f"[graphs] {case}: calls of 21, 8, 3 and 16 steps")
    bs = CASES[case]()
    ctxs = [A.context_for(bs, e) for e in (A.EXEC_BATCHED, A.EXEC_PER_BLOCK)]
    try:
        for n in (21, 8, 3, 16):
            ts = [ctx.ssprk_step(oracle.SSPRK54, n, cfl=0.4, t=0.0) for ctx, _, _ in ctxs]
            scratch = torch.ones(1 << 16, dtype=torch.float64, device="cuda").cumsum(0)   # eager work between
            torch.cuda.synchronize()
            del scratch
            assert ts[0] == ts[1]
            assert torch.equal(ctxs[0][1], ctxs[1][1])
    finally:
        for ctx, _, _ in ctxs:
            ctx.close()


def test_runs_are_bitwise_deterministic():
    bs = CASES["mhd3d"]()
    say("[determinism] mhd3d")
    a, ta = gpu_run(bs, oracle.SSPRK54, 5)
    b, tb = gpu_run(bs, oracle.SSPRK54, 5)
    assert ta == tb
    for x, y in zip(a.u, b.u):
        assert np.array_equal(x, y)


def test_block_decomposition_is_bitwise_invisible():
    say("[decomposition] ot2d 1 block vs 16 blocks")
    one = inputs.orszag_tang_2d(64, 64)
    many = inputs.orszag_tang_2d(64, 16)
    a, ta = gpu_run(one, oracle.SSPRK54, 10)
    b, tb = gpu_run(many, oracle.SSPRK54, 10)
    assert ta == tb
    ua = a.interior(0)
    for blk in range(many.nb):
        ox = int(round(many.xlo[blk, 0] * 64))
        oy = int(round(many.xlo[blk, 1] * 64))
        assert np.array_equal(ua[:, :, oy:oy + 16, ox:ox + 16], b.interior(blk))


def test_periodic_conservation_on_gpu():
    say("[conservation] mhd3d 20 steps")
    bs = CASES["mhd3d"]()
    out, _ = gpu_run(bs, oracle.SSPRK54, 20)
    for v in range(bs.nvar):
        t0 = math.fsum(float(x) for b in range(bs.nb) for x in bs.interior(b)[v].ravel())
        t1 = math.fsum(float(x) for b in range(bs.nb) for x in out.interior(b)[v].ravel())
        scale = math.fsum(abs(float(x)) for b in range(bs.nb) for x in bs.interior(b)[v].ravel())
        assert abs(t1 - t0) <= 1e-13 * max(scale, 1.0), (v, t0, t1)


def test_free_stream_is_bitwise_uniform_on_gpu():
    say("[free stream] 3D MHD")
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(3, [16, 16, 16], [8, 8, 8])
    w = {"rho": 1.3, "p": 0.7, "vx": 0.4, "vy": -0.3, "vz": 0.2, "Bx": 0.9, "By": -0.5, "Bz": 0.25}
    bs = inputs.sample_blocks(3, True, 5 / 3, n, dx, xlo, nbr,
                              lambda X, Y, Z: {k: v + 0 * X for k, v in w.items()})
    Lg, _ = gpu_rhs(bs)
    for L in Lg:
        assert np.all(L == 0.0)
    out, _ = gpu_run(bs, oracle.SSPRK54, 3)
    ref = out.interior(0)[:, 0, 0, 0]
    for b in range(bs.nb):
        assert np.all(out.interior(b) == ref[:, None, None, None])


def test_nonphysical_state_is_reported():
    say("[error] negative pressure")
    bs = inputs.sod(64)
    bs.interior(0)[2, 0, 0, 10] = -1.0     # E < 0 -> p < 0
    ctx, flat, views = A.context_for(bs)
    with pytest.raises(A.AmrvacError) as ei:
        ctx.ssprk_step(oracle.SSPRK54, 1, t=0.0)
    assert ei.value.status == A.ERR_NONPHYSICAL
    ctx.sync()   # the flag was cleared by the report
    ctx.close()


def test_invalid_arguments_leave_state_untouched():
    bs = inputs.orszag_tang_2d(32, 16)
    ctx, flat, views = A.context_for(bs)
    before = flat.clone()
    with pytest.raises(A.AmrvacError) as ei:
        ctx.ssprk_step(7, 1)
    assert ei.value.status == A.ERR_INVALID
    with pytest.raises(A.AmrvacError):
        ctx.ssprk_step(oracle.SSPRK54, 1, cfl=-1.0)
    with pytest.raises(A.AmrvacError):
        ctx.ssprk_step(oracle.SSPRK54, 1, dt=float("nan"))
    torch.cuda.synchronize()
    assert torch.equal(before, flat)
    ctx.close()


def test_zero_steps_leave_state_and_time_untouched():
    say("[edge] nsteps = 0, every execution form and every scheme")
    bs = uneven_small()
    ctx, flat, views = A.context_for(bs)
    before = flat.clone()
    for exec in (A.EXEC_BATCHED, A.EXEC_PER_BLOCK, A.EXEC_BATCHED_SINGLE):
        ctx.set_exec(exec)
        for scheme in (oracle.RK3, oracle.SSPRK43, oracle.SSPRK54):
            assert ctx.ssprk_step(scheme, 0, t=0.125) == 0.125
            assert ctx.ssprk_step(scheme, 0, dt=1e-3, t=0.25) == 0.25
    torch.cuda.synchronize()
    assert torch.equal(before, flat)
    ctx.close()


# ---------------------------------------------------------------- full sizes
def test_full_size_2d_mhd_rhs_and_100_steps():
    """512^2 as 1024 blocks of 16^2 (the 2D MHD workload), right-hand side
    element by element and the state after 100 SSPRK(5,4) steps."""
    say("[full] 2D MHD 512^2 rhs")
    bs = inputs.orszag_tang_2d(512, 16)
    Lo, cmo = oracle.rhs(bs)
    Lg, cmg = gpu_rhs(bs)
    np.testing.assert_allclose(cmg, cmo, rtol=1e-14)
    compare_rhs(bs, Lg, Lo, cmo)
    say("[full] 2D MHD 512^2 100 steps (oracle on host cores)")
    out_o, dts = oracle.run(bs, oracle.SSPRK54, 100)
    out_g, t = gpu_run(bs, oracle.SSPRK54, 100)
    assert abs(t - dts.sum()) <= 1e-12 * dts.sum()
    assert_state_parity(bs, out_g, out_o)


def sample_blocks_with_true_ghosts(bs, idx):
    """Sub-list of blocks whose ghost layers (sampled from the same periodic
    lattice) are used as fixed faces: L of each block then equals its L in
    the full list given the full list's c_max."""
    sub = bs.copy()
    sub.u = [bs.u[i] for i in idx]
    sub.n = bs.n[idx].copy()
    sub.dx = bs.dx[idx].copy()
    sub.xlo = bs.xlo[idx].copy()
    sub.nbr = -np.ones((len(idx), 6), np.int32)
    return sub


@pytest.mark.parametrize("which", ["uneven3d_4096", "mhd3d_256"])
def test_full_size_3d_rhs_on_sampled_blocks(which):
    say(f"[full] {which} rhs, sampled blocks")
    bs = inputs.uneven_3d() if which == "uneven3d_4096" else inputs.mhd_turbulence_3d()
    Lg, cmg = gpu_rhs(bs)
    cmo = oracle.cmax(bs)
    np.testing.assert_allclose(cmg, cmo, rtol=1e-14)
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.choice(bs.nb, 24, replace=False), [0, bs.nb - 1]]))
    sub = sample_blocks_with_true_ghosts(bs, idx)
    Lo, _ = oracle.rhs(sub, cmax=cmo)
    compare_rhs(sub, [Lg[i] for i in idx], Lo, cmo)


def test_full_size_uneven3d_10_steps_in_bench_configuration():
    """The 4096-block uneven 3D MHD list in the configuration bench.py times
    (autotuned tile shape, batched persistent launch, one graph per step):
    10 SSPRK(5,4) steps are bitwise equal to the per-block launch form, and
    the right-hand side of the state they reach matches the oracle on
    sampled blocks."""
    say("[full] uneven3d 4096 blocks: autotune + 10 batched steps")
    bs = inputs.uneven_3d()
    ctx, flat, views = A.context_for(bs, A.EXEC_BATCHED)
    ctx.autotune(oracle.SSPRK54, 1)
    t_b = ctx.ssprk_step(oracle.SSPRK54, 10, cfl=0.4, t=0.0)
    out = bs.copy()
    out.u = host_blocks(views)
    ctx.close()
    say("[full] uneven3d 4096 blocks: 10 per-block steps")
    ref, t_p = gpu_run(bs, oracle.SSPRK54, 10, exec=A.EXEC_PER_BLOCK)
    assert t_b == t_p
    for x, y in zip(out.u, ref.u):
        assert np.array_equal(x, y)
    say("[full] uneven3d 4096 blocks: 10 steps, one launch per stage over the whole list")
    one, t_s = gpu_run(bs, oracle.SSPRK54, 10, exec=A.EXEC_BATCHED_SINGLE)
    assert t_s == t_p
    for x, y in zip(one.u, ref.u):
        assert np.array_equal(x, y)
    say("[full] uneven3d 4096 blocks: rhs of the stepped state, sampled blocks")
    Lg, cmg = gpu_rhs(out)
    cmo = oracle.cmax(out)
    np.testing.assert_allclose(cmg, cmo, rtol=1e-14)
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([rng.choice(out.nb, 24, replace=False), [0, out.nb - 1]]))
    sub = sample_blocks_with_true_ghosts(out, idx)
    Lo, _ = oracle.rhs(sub, cmax=cmo)
    compare_rhs(sub, [Lg[i] for i in idx], Lo, cmo)


def test_full_size_mhd3d_256_conserves_totals():
    """256^3 periodic 3D MHD (4096 blocks of 16^3): after 10 batched
    SSPRK(5,4) steps the totals of all eight conserved variables equal their
    initial totals to rounding (the scheme is conservative and the grid is
    periodic)."""
    say("[full] mhd3d 256^3: 10 steps, conserved totals")
    bs = inputs.mhd_turbulence_3d()
    tot0 = [math.fsum(float(bs.interior(b)[v].sum()) for b in range(bs.nb)) for v in range(bs.nvar)]
    mag = [math.fsum(float(np.abs(bs.interior(b)[v]).sum()) for b in range(bs.nb)) for v in range(bs.nvar)]
    out, _ = gpu_run(bs, oracle.SSPRK54, 10)
    tot1 = [math.fsum(float(out.interior(b)[v].sum()) for b in range(out.nb)) for v in range(out.nvar)]
    for v in range(bs.nvar):
        assert abs(tot1[v] - tot0[v]) <= 1e-12 * mag[v], (v, tot0[v], tot1[v], mag[v])


# ---------------------------------------------------------------- tile shapes
@pytest.mark.parametrize("case", ["dwave1d_8blk", "ot2d", "hydro2d", "ragged2d_mhd", "mhd3d", "uneven3d",
                                  "ragged3d_hd", "ragged3d_mhd", "min3_3d_mhd", "min3_1d_mhd"])
def test_every_tile_shape_is_bitwise_identical(case):
    bs = CASES[case]()
    ref = None
    ctx0, _, _ = A.context_for(bs)
    names = ctx0.variants()
    ctx0.close()
    for i, name in enumerate(names):
        say(f"[variant] {case} {name}")
        ctx, flat, views = A.context_for(bs)
        ctx.set_variant(i)
        t = ctx.ssprk_step(oracle.SSPRK54, 3, t=0.0)
        got = host_blocks(views), t
        ctx.close()
        if ref is None:
            ref = got
            continue
        assert got[1] == ref[1], name
        for x, y in zip(got[0], ref[0]):
            assert np.array_equal(x, y), name


def test_autotune_reads_but_never_writes_the_state():
    say("[autotune] mhd3d")
    bs = CASES["mhd3d"]()
    ctx, flat, views = A.context_for(bs)
    before = flat.clone()
    name, ms = ctx.autotune(oracle.SSPRK54, 1)
    torch.cuda.synchronize()
    assert torch.equal(before, flat)
    assert name in ctx.variants()
    timed = [m for m in ms if m >= 0]
    assert timed and min(timed) == ms[ctx.variants().index(name)]
    out_o, _ = oracle.run(bs, oracle.SSPRK54, 5)
    t = ctx.ssprk_step(oracle.SSPRK54, 5, t=0.0)
    out_g = bs.copy()
    out_g.u = host_blocks(views)
    ctx.close()
    assert_state_parity(bs, out_g, out_o)
