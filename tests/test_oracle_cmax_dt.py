"""Pins of the oracle's global c_max (Sect. 2.2: the grid-global maximal
characteristic velocity of the Lax-Friedrichs split, reading: per direction,
over the interior cells of every block) and of its time step (the multi-D
form of the bound dt < dx / c_w of Sect. 4.4).

Independent of the oracle's own formulas: the characteristic speed of a cell
along d is taken as the spectral radius of the flux Jacobian dF_d/dU, built
by central differences of the flux and handed to numpy's eigenvalue solver
(for hydro and ideal MHD it equals |v_d| + c_f,d).  The cases put mixed-sign
velocities in the interior, a different fastest cell per direction, and much
faster states in the ghost layers, which must not enter the maximum."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs


def spectral_radius(ndim, mhd, gamma, d, u):
    n = len(u)
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * max(1.0, abs(u[j]))
        e = np.zeros(n)
        e[j] = h
        J[:, j] = (oracle.flux(ndim, mhd, gamma, d, u + e) - oracle.flux(ndim, mhd, gamma, d, u - e)) / (2 * h)
    return float(np.abs(np.linalg.eigvals(J)).max())


def isolated_blocks(ndim, mhd, gamma, ns, dxs, seed, ghost_boost=0.0):
    """Blocks with fixed faces, random smooth primitives with both signs of
    every velocity component; ghost cells get |v| raised by ghost_boost."""
    rng = np.random.default_rng(seed)
    nb = len(ns)
    n = np.ones((nb, 3), np.int32)
    dx = np.ones((nb, 3))
    xlo = np.zeros((nb, 3))
    nbr = -np.ones((nb, 6), np.int32)
    for b in range(nb):
        n[b, :ndim] = ns[b][:ndim]
        dx[b, :ndim] = dxs[b][:ndim]
    amp = {k: rng.uniform(0.2, 0.6) for k in ("vx", "vy", "vz", "Bx", "By", "Bz")}
    ph = {k: rng.uniform(0, 2 * math.pi, size=3) for k in amp}

    def f(X, Y, Z):
        shape = np.broadcast_shapes(X.shape, Y.shape, Z.shape)
        out = {"rho": 1.0 + 0.3 * np.sin(2 * math.pi * (X + 2 * Y) + 0.3) + 0 * X,
               "p": 0.8 + 0.4 * np.cos(2 * math.pi * (2 * X - Y + Z)) + 0 * X}
        for k in amp:
            out[k] = amp[k] * np.sin(2 * math.pi * X + ph[k][0]) * np.cos(2 * math.pi * Y + ph[k][1]) + \
                0.5 * amp[k] * np.sin(2 * math.pi * Z + ph[k][2]) + 0 * X
        return {k: np.broadcast_to(v, shape) for k, v in out.items()}
    bs = inputs.sample_blocks(ndim, mhd, gamma, n, dx, xlo, nbr, f)
    if ghost_boost:
        nc = 3 if mhd else ndim
        for b in range(nb):
            ghost = np.ones(bs.u[b].shape[1:], dtype=bool)
            bs.interior(b, ghost[None])[...] = False
            for k in range(nc):   # momentum += rho * boost in the ghosts (kinetic energy too)
                m = bs.u[b][1 + k]
                rho = bs.u[b][0]
                dm = np.where(ghost, rho * ghost_boost * (1 if k % 2 == 0 else -1), 0.0)
                ie = 1 + nc
                bs.u[b][ie] = bs.u[b][ie] + (m * dm + 0.5 * dm * dm) / rho
                bs.u[b][1 + k] = m + dm
    return bs


def independent_cmax(bs):
    cm = np.zeros(3)
    for b in range(bs.nb):
        x = bs.interior(b)
        flat = x.reshape(bs.nvar, -1)
        for c in range(flat.shape[1]):
            u = flat[:, c].copy()
            for d in range(bs.ndim):
                cm[d] = max(cm[d], spectral_radius(bs.ndim, bs.mhd, bs.gamma, d, u))
    return cm


CASES = [
    ("hydro1d", 1, False, 1.4, [(9,), (6,)]),
    ("hydro2d", 2, False, 1.4, [(6, 5), (4, 7)]),
    ("mhd2d", 2, True, 5 / 3, [(6, 5), (5, 4)]),
    ("mhd3d", 3, True, 5 / 3, [(4, 3, 5), (3, 4, 3)]),
]


@pytest.mark.parametrize("case,ndim,mhd,gamma,ns", CASES, ids=[c[0] for c in CASES])
def test_cmax_is_per_direction_max_over_interior_cells(case, ndim, mhd, gamma, ns):
    dxs = [(1.0 / 16, 1.0 / 12, 1.0 / 10)] * len(ns)
    bs = isolated_blocks(ndim, mhd, gamma, ns, dxs, seed=len(case), ghost_boost=3.0)
    exp = independent_cmax(bs)
    got = oracle.cmax(bs)
    np.testing.assert_allclose(got[:ndim], exp[:ndim], rtol=1e-7)
    assert np.all(got[ndim:] == 0.0)
    # the maximum is per direction: the directions' maxima differ here
    if ndim > 1:
        assert abs(exp[0] - exp[1]) > 1e-3 * exp[0]
    # the ghosts are much faster (|v| raised by 3): a maximum that read them
    # would exceed the interior one by far
    assert max(float(np.abs(bs.u[b][1:1 + (3 if mhd else ndim)] / bs.u[b][0]).max())
               for b in range(bs.nb)) > 2.0
    # c_max returned by the right-hand side is the same maximum
    _, cm_rhs = oracle.rhs(bs)
    np.testing.assert_array_equal(cm_rhs, got)


def test_cmax_uses_the_magnitude_of_negative_velocities():
    """One cell moving fast in -x sets c_max,x; |v_x| enters, not v_x."""
    bs = isolated_blocks(1, False, 1.4, [(8,)], [(0.1,)], seed=3)
    rho = bs.interior(0)[0].copy()
    c = 5
    bs.interior(0)[1, 0, 0, c] = -4.0 * rho[0, 0, c]
    bs.interior(0)[2, 0, 0, c] += 0.5 * 16.0 * rho[0, 0, c]   # E += rho v^2 / 2 keeps p
    exp = independent_cmax(bs)
    got = oracle.cmax(bs)
    assert got[0] > 4.0
    np.testing.assert_allclose(got[0], exp[0], rtol=1e-7)


def test_time_step_of_the_density_wave():
    """1D Euler density wave rho = 1 + 0.2 sin(2 pi x), v = 1, p = 1, gamma
    1.4, 512 cells, Courant 0.4: dt = 0.4 dx / (1 + sqrt(gamma p / rho_min))
    with rho_min the smallest sampled density, the bound dt < dx / c_w of
    Sect. 4.4 at the Courant number 0.4 of the paper's FD runs."""
    bs = inputs.density_wave_1d(512)
    x = (np.arange(512) + 0.5) / 512
    rho_min = float((1.0 + 0.2 * np.sin(2 * math.pi * x)).min())
    exp = 0.4 * (1.0 / 512) / (1.0 + math.sqrt(1.4 / rho_min))
    _, dts = oracle.run(bs, oracle.RK3, 1, cfl=0.4)
    assert abs(dts[0] - exp) <= 1e-13 * exp, (dts[0], exp)
    # the rounded value of the configuration: 0.4 (1/512) / (1 + sqrt(1.75))
    assert abs(dts[0] - 0.4 / 512 / (1 + math.sqrt(1.75))) < 1e-4 * dts[0]


@pytest.mark.parametrize("ndim,mhd", [(2, False), (2, True), (3, True)])
def test_multi_d_time_step_is_worst_block_of_sum_over_directions(ndim, mhd):
    """dt = CFL / max over blocks of sum_d c_max,d / dx_d, with c_max,d the
    global maxima: blocks of different cell widths, the finest decides."""
    ns = [(4, 5, 3), (5, 4, 4), (3, 3, 5)]
    dxs = [(1 / 8, 1 / 10, 1 / 6), (1 / 20, 1 / 7, 1 / 9), (1 / 12, 1 / 30, 1 / 5)]
    bs = isolated_blocks(ndim, mhd, 5 / 3 if mhd else 1.4, ns, dxs, seed=7 + ndim)
    cm = independent_cmax(bs)
    worst = max(sum(cm[d] / dxs[b][d] for d in range(ndim)) for b in range(len(ns)))
    exp = 0.3 / worst
    _, dts = oracle.run(bs, oracle.SSPRK54, 1, cfl=0.3)
    assert abs(dts[0] - exp) <= 1e-7 * exp, (dts[0], exp)
    # a single block's sum would differ: the maximum over blocks matters
    sums = [sum(cm[d] / dxs[b][d] for d in range(ndim)) for b in range(len(ns))]
    assert max(sums) > 1.2 * min(sums)


def test_time_step_is_recomputed_each_step_from_the_step_state():
    """dt of step 2 is the rule applied to U^1 (not to U^0)."""
    bs = inputs.sod(64)
    out1, dts = oracle.run(bs, oracle.SSPRK54, 2, cfl=0.4)
    one, d1 = oracle.run(bs, oracle.SSPRK54, 1, cfl=0.4)
    cm = independent_cmax(one)
    exp = 0.4 / (cm[0] / bs.dx[0, 0])
    assert abs(dts[1] - exp) <= 1e-7 * exp
    assert dts[1] != dts[0]
