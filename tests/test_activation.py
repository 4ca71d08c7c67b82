"""Dynamic grid activation (the paper's appendix "Dynamic grid activation"):
the host-side list building of the library against a plain breadth-first
reference, and the oracle's masked integration pinned to its unmasked one.
CPU only."""
import numpy as np
import pytest

import oracle
from helpers import smooth_fields
from paper_1407_2052_amd import amrvac as A
from paper_1407_2052_amd import inputs


def belt_reference(nbr, want, safety):
    """Steps 1-2 of the appendix: flag, then `safety` passes that re-activate
    every passive block with an active face neighbour."""
    cur = [bool(w) for w in want]
    for _ in range(safety):
        nxt = list(cur)
        for b in range(len(cur)):
            if not cur[b] and any(nb >= 0 and cur[nb] for nb in nbr[b]):
                nxt[b] = True
        cur = nxt
    return np.array(cur, dtype=np.uint8)


@pytest.mark.parametrize("ndim,grid,periodic", [(1, [12], True), (2, [6, 5], True), (2, [6, 5], False),
                                                (3, [4, 3, 5], True)])
def test_safety_belt_matches_reference(ndim, grid, periodic):
    N = [8 * g for g in grid]
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(ndim, N, [8] * ndim)
    if not periodic:
        # cut the periodic wrap: faces on the domain boundary become fixed
        for b in range(len(n)):
            for d in range(ndim):
                i = int(round(xlo[b, d] / dx[b, d])) // 8
                if i == 0:
                    nbr[b, 2 * d] = -1
                if i == grid[d] - 1:
                    nbr[b, 2 * d + 1] = -1
    rng = np.random.default_rng(ndim * 7 + periodic)
    for safety in range(4):
        for trial in range(5):
            want = rng.random(len(n)) < 0.15
            cnt, got = A.activation_flags(nbr, want, safety)
            ref = belt_reference(nbr, want, safety)
            assert np.array_equal(got, ref), (safety, trial)
            assert cnt == int(ref.sum())


def test_activation_flags_rejects_invalid_arguments():
    nbr = np.array([[1, 1, -1, -1, -1, -1], [0, 0, -1, -1, -1, -1]])
    assert A.activation_flags(nbr, [1, 0], -1)[0] == -1
    bad = nbr.copy()
    bad[0, 0] = 5
    assert A.activation_flags(bad, [1, 0], 1)[0] == -1
    bad[0, 0] = -2
    assert A.activation_flags(bad, [1, 0], 1)[0] == -1
    assert A.activation_flags(nbr, [0, 0], 3) == (0, pytest.approx(np.zeros(2)))


def island_grid(seed=2):
    """2D MHD on 8 x 8 periodic blocks of 16^2: a smooth perturbation inside
    one block (cells away from its faces) on an exactly uniform background,
    which is a stationary solution of the scheme (free stream)."""
    N, B = 128, 16
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(2, [N, N], [B, B])
    f = smooth_fields(2, True, seed, amp=0.05)
    back = {"rho": 1.0, "vx": 0.3, "vy": -0.2, "vz": 0.1, "p": 1.0, "Bx": 0.8, "By": 0.4, "Bz": -0.3}
    cx = cy = (4 * B + 8) / N

    def fields(X, Y, Z):
        # perturbation inside the centre block only (radius 5 cells), exactly
        # the uniform background elsewhere
        r2 = ((X - cx) ** 2 + (Y - cy) ** 2) * (N / 5.0) ** 2
        w = np.where(r2 < 1.0, np.exp(-r2), 0.0)
        pert = f(X, Y, Z)
        return {k: back[k] + w * (pert[k] - back[k]) for k in back}
    return inputs.sample_blocks(2, True, 5 / 3, n, dx, xlo, nbr, fields)


def test_stationary_passive_region_equals_the_all_active_run():
    """Blocks far from the perturbation hold a free stream (L = 0 exactly).
    Made passive behind a safety belt wider than the numerical domain of
    dependence of the run (3 cells per stage), they must not change the
    result: the masked run equals the all-active run bitwise, interiors and
    time steps alike."""
    bs = island_grid()
    centre = [b for b in range(bs.nb) if abs(bs.xlo[b, 0] - 0.5) < 1e-12 and abs(bs.xlo[b, 1] - 0.5) < 1e-12]
    assert len(centre) == 1
    want = np.zeros(bs.nb, bool)
    want[centre[0]] = True
    _, flags = A.activation_flags(bs.nbr, want, 2)
    ref, dts_ref = oracle.run(bs, oracle.SSPRK54, 1, cfl=0.4)
    oracle.set_active(flags)
    try:
        got, dts = oracle.run(bs, oracle.SSPRK54, 1, cfl=0.4)
    finally:
        oracle.set_active(None)
    assert np.array_equal(dts, dts_ref)
    for b in range(bs.nb):
        assert np.array_equal(got.interior(b), ref.interior(b)), b
        if not flags[b]:
            assert np.array_equal(got.interior(b), bs.interior(b))


def test_passive_blocks_keep_their_state_and_feed_neighbours():
    bs = inputs.orszag_tang_2d(64, 16)
    flags = np.ones(bs.nb, np.uint8)
    flags[[0, 5, 10]] = 0
    oracle.set_active(flags)
    try:
        out, _ = oracle.run(bs, oracle.SSPRK54, 3)
        L, _ = oracle.rhs(bs)
    finally:
        oracle.set_active(None)
    full, _ = oracle.run(bs, oracle.SSPRK54, 3)
    for b in range(bs.nb):
        if flags[b]:
            assert not np.array_equal(out.interior(b), bs.interior(b))
        else:
            assert np.array_equal(out.interior(b), bs.interior(b))
            assert not np.any(bs.interior(b, L[b]))
    # the frozen neighbours change their active neighbours' evolution
    assert any(not np.array_equal(out.interior(b), full.interior(b)) for b in (1, 4))
