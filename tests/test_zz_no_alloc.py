"""amrvac_ssprk_step_noalloc (through the C ABI) against amrvac_ssprk_step:
the same kernels on stage buffers in the library's fixed device array, so
the results must agree bit for bit (a stronger bar than the oracle parity
of the stepping itself).  Two calls in a row, the second on a smaller block
list, so the second reads nothing the first left behind; a block list too
large for the array is refused before anything runs."""
import sys

import numpy as np
import pytest

import oracle
from helpers import strip_blocks
from paper_1407_2052_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1407_2052_amd import amrvac as A  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(bs, scheme, nsteps, noalloc, exec=A.EXEC_BATCHED, dt=None):
    ctx, flat, views = A.context_for(bs, exec)
    step = ctx.ssprk_step_noalloc if noalloc else ctx.ssprk_step
    t = step(scheme, nsteps, cfl=0.4, dt=dt, t=0.0)
    out = [v.detach().cpu().numpy() for v in views]
    ctx.close()
    return out, t


def assert_same(bs, scheme, nsteps, exec=A.EXEC_BATCHED, dt=None):
    got, tg = run(bs, scheme, nsteps, True, exec, dt)
    ref, tr = run(bs, scheme, nsteps, False, exec, dt)
    assert tg == tr
    for b, (x, y) in enumerate(zip(got, ref)):
        assert np.array_equal(x, y), b
    # and the state did advance
    assert any(not np.array_equal(x, y) for x, y in zip(got, bs.u))


def test_two_calls_in_a_row_second_smaller_equal_ssprk_step():
    say("[noalloc] 2D MHD 64^2 in 16^2 blocks, 10 SSPRK(5,4) steps")
    big = inputs.orszag_tang_2d(64, 16)
    assert 3 * big.interior_cells() * big.nvar <= A.NOALLOC_MAX_DOUBLES
    assert_same(big, oracle.SSPRK54, 10)
    say("[noalloc] 1D Euler 512 in 4 blocks, 20 RK3 steps (smaller)")
    small = inputs.density_wave_1d(512, nblocks=4)
    assert small.interior_cells() * small.nvar < big.interior_cells() * big.nvar
    assert_same(small, oracle.RK3, 20)


def test_fixed_faces_both_execution_forms_and_fixed_dt():
    say("[noalloc] 3D MHD uneven blocks with fixed faces, SSPRK(5,4), both execution forms")
    bs = inputs.uneven_3d(nblocks=14, seed=3, N=64)
    assert_same(bs, oracle.SSPRK54, 4, A.EXEC_BATCHED)
    assert_same(bs, oracle.SSPRK54, 4, A.EXEC_PER_BLOCK)
    say("[noalloc] ragged 2D hydro, SSPRK(4,3) at a fixed dt")
    rg = strip_blocks(2, False, [13, 19, 7], ny=10, seed=1, gamma=1.4)
    assert_same(rg, oracle.SSPRK43, 6, dt=1e-3)


def test_matches_the_oracle():
    say("[noalloc] 2D Euler 64^2 vs oracle, 50 SSPRK(5,4) steps")
    bs = inputs.hydro_random_2d(64, 16, seed=4)
    got, t = run(bs, oracle.SSPRK54, 50, True)
    ref, dts = oracle.run(bs, oracle.SSPRK54, 50, cfl=0.4)
    assert abs(t - dts.sum()) <= 1e-12 * dts.sum()
    for v in range(bs.nvar):
        num = sum(float(np.abs(bs.interior(b, got[b])[v] - ref.interior(b)[v]).sum()) for b in range(bs.nb))
        den = sum(float(np.abs(ref.interior(b)[v]).sum()) for b in range(bs.nb))
        assert (num == 0.0) if den == 0.0 else (num / den <= 1e-11), (v, num, den)


def test_too_large_block_list_is_refused_without_touching_the_state():
    say("[noalloc] 96^3 MHD: stage buffers larger than the fixed array")
    bs = inputs.mhd_turbulence_3d(N=96, block=16, seed=5)
    assert 3 * bs.interior_cells() * bs.nvar > A.NOALLOC_MAX_DOUBLES
    ctx, flat, views = A.context_for(bs)
    before = flat.clone()
    with pytest.raises(A.AmrvacError) as ei:
        ctx.ssprk_step_noalloc(oracle.SSPRK54, 1, t=0.0)
    assert ei.value.status == A.ERR_INVALID
    torch.cuda.synchronize()
    assert torch.equal(before, flat)
    # the context still steps through its own scratch
    ctx.ssprk_step(oracle.SSPRK54, 1, t=0.0)
    ctx.close()
