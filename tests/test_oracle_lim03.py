"""Pins of the oracle's LIM03 reconstruction (Cada & Torrilhon 2009, offered
beside MP5 in Sect. 2.2): exactness on polynomials, the asymptotic-region
switch, limiting at steps and extrema, symmetries, the derivative of the
branch taken, and the scheme-level results the paper prints for RK3 + LIM03
(third order in both norms on the Alfven wave, Sect. 4.5.1; no contact
overshoot in the Brio-Wu tube, Sect. 4.5.2)."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs
from test_oracle_mp5 import cell_average
from test_oracle_solutions import fixed_dt, paper_number, run_to_time, total


@pytest.fixture(autouse=True)
def lim03_radius_default():
    yield
    oracle.set_lim03_radius(1.0)


# --------------------------------------------------------------- single reconstruction
@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("amp", [1e-3, 1e3])
def test_exact_for_monotone_quadratic_cell_averages(seed, amp):
    # amp 1e-3: eta <= 1 (asymptotic branch); amp 1e3: eta > 1 with theta in
    # the range where the limited function equals the unlimited one.
    rng = np.random.default_rng(seed)
    h = 0.05
    c = amp * np.array([0.3, 1.0, rng.uniform(-2.0, 2.0)])
    x0 = rng.uniform(-0.05, 0.05)
    f = [cell_average(c, x0 + (j - 0.5) * h, x0 + (j + 0.5) * h) for j in (-1, 0, 1)]
    dm, dp = f[1] - f[0], f[2] - f[1]
    assert dp != 0.0 and 0.4 < dm / dp < 2.8
    exact = np.polynomial.polynomial.polyval(x0 + 0.5 * h, c)
    assert abs(oracle.lim03(f, h) - exact) < 1e-13 * amp


@pytest.mark.parametrize("seed", range(6))
def test_fd_derivative_exact_for_cubic_point_values(seed):
    # Conservative FD derivative (Sect. 2.1) from the third-order
    # reconstruction: exact for point values of a polynomial of degree <= 3.
    rng = np.random.default_rng(200 + seed)
    h = 0.02
    c = np.array([0.1, 0.02 * rng.uniform(-1, 1), *rng.uniform(-0.4, 0.4, size=2)])
    xi = rng.uniform(-0.3, 0.3)
    pts = [np.polynomial.polynomial.polyval(xi + j * h, c) for j in range(-2, 2)]
    right = oracle.lim03(pts[1:4], h)
    left = oracle.lim03(pts[0:3], h)
    deriv = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(c))
    assert abs((right - left) / h - deriv) < 1e-10


def test_asymptotic_switch_keeps_smooth_extrema_and_limits_large_ones():
    # Smooth maximum: the limited function alone clips the slope (theta in
    # (-0.8, 0)); inside the asymptotic region the third-order value stays.
    h = 0.01
    f = np.array([math.cos((j + 0.3) * h) for j in (-1, 0, 1)]) * 1e-3
    third = (-f[0] + 5 * f[1] + 2 * f[2]) / 6
    theta = (f[1] - f[0]) / (f[2] - f[1])
    assert -0.8 < theta < 0.0
    assert oracle.lim03(f, h) == pytest.approx(third, rel=0, abs=1e-18)
    # the same shape with eta > 1 is limited: phi = -theta/2
    oracle.set_lim03_radius(1e-9)
    lim = f[1] + 0.5 * (-0.5 * theta) * (f[2] - f[1])
    assert oracle.lim03(f, h) == pytest.approx(lim, rel=1e-14)
    assert abs(oracle.lim03(f, h) - third) > 1e-9


@pytest.mark.parametrize("scale", [1.0, 1e6])
def test_steps_produce_no_overshoot(scale):
    for f in ([0, 0, 1], [0, 1, 1], [1, 1, 0], [1, 0, 0], [0, 0, 0], [1, 0, 1]):
        a = scale * np.array(f, float)
        r = oracle.lim03(a, 1e-3)
        lo, hi = min(a[1], a[2]), max(a[1], a[2])
        assert lo <= r <= hi or (a[0] == a[2] and abs(r - a[1]) <= 0.25 * abs(a[1] - a[0]))


def test_large_monotone_data_stays_between_centre_and_neighbour():
    rng = np.random.default_rng(5)
    for _ in range(20000):
        f = np.sort(rng.normal(size=3)) * rng.choice([-1.0, 1.0]) * 1e3
        r = oracle.lim03(f, 1e-3)
        assert min(f[1], f[2]) <= r <= max(f[1], f[2])


def test_large_extremum_moves_at_most_a_quarter_of_the_upwind_jump():
    # theta < 0 outside the asymptotic region: phi <= -theta/2, so the
    # interface value differs from f_j by at most |f_j - f_{j-1}| / 4.
    rng = np.random.default_rng(9)
    for _ in range(5000):
        a, c = rng.normal(size=2) * 1e3
        b = max(a, c) + abs(rng.normal()) * 1e3
        r = oracle.lim03([a, b, c], 1e-3)
        # equality on the -theta/2 piece; rounding of f_j + H/2 is ulp(f_j)
        assert abs(r - b) <= 0.25 * abs(b - a) + 4e-16 * abs(b)


@pytest.mark.parametrize("seed", range(3))
def test_odd_symmetry_and_power_of_two_scaling_bitwise(seed):
    rng = np.random.default_rng(seed)
    for _ in range(3000):
        f = rng.normal(size=3) * 10.0 ** rng.uniform(-4, 2)
        h = 10.0 ** rng.uniform(-3, -1)
        r = oracle.lim03(f, h)
        assert oracle.lim03(-f, h) == -r
        # eta is invariant when the data and the cell width scale together
        assert oracle.lim03(4.0 * f, 4.0 * h) == 4.0 * r
        assert oracle.lim03(0.125 * f, 0.125 * h) == 0.125 * r


def test_constant_data():
    for v in (0.0, 0.5, -3.25, 2.5e8):
        assert oracle.lim03([v] * 3, 0.01) == v


def test_gradient_of_branch_taken_matches_differences():
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(3000):
        f = rng.normal(size=3) * 10.0 ** rng.uniform(-3, 1)
        h = 0.05
        v, g = oracle.lim03_grad(f, h)
        assert v == oracle.lim03(f, h)
        eps = 1e-8 * max(1e-3, np.abs(f).max())
        fd = np.zeros(3)
        for i in range(3):
            e = np.zeros(3); e[i] = eps
            fd[i] = (oracle.lim03(f + e, h) - oracle.lim03(f - e, h)) / (2 * eps)
        if np.max(np.abs(fd - g)) < 1e-5:
            checked += 1
    assert checked > 2900


def test_gradients_of_the_linear_pieces():
    # asymptotic region and the unlimited piece: (-1, 5, 2)/6
    _, g = oracle.lim03_grad([1e-4, 2e-4, 3e-4], 0.01)
    np.testing.assert_allclose(g * 6.0, [-1, 5, 2], atol=1e-12)
    _, g = oracle.lim03_grad([0.0, 1.0, 2.0], 1e-3)
    np.testing.assert_allclose(g * 6.0, [-1, 5, 2], atol=1e-12)
    # cap phi = 1.6: f_j + 0.8 (f_{j+1} - f_j)
    _, g = oracle.lim03_grad([0.0, 10.0, 11.0], 1e-3)
    np.testing.assert_allclose(g, [0.0, 0.2, 0.8], atol=1e-12)
    # TVD bound phi = 2 theta: 2 f_j - f_{j-1}
    _, g = oracle.lim03_grad([0.0, 1.0, 11.0], 1e-3)
    np.testing.assert_allclose(g, [-1.0, 2.0, 0.0], atol=1e-12)
    # extremum phi = -theta/2: (f_{j-1} + 3 f_j) / 4
    _, g = oracle.lim03_grad([9.0, 10.0, 1.0], 1e-3)
    np.testing.assert_allclose(g, [0.25, 0.75, 0.0], atol=1e-12)
    # extremum with theta < -0.8: the unlimited piece again
    _, g = oracle.lim03_grad([0.0, 10.0, 1.0], 1e-3)
    np.testing.assert_allclose(g * 6.0, [-1, 5, 2], atol=1e-12)
    # flat upwind side: f_j
    _, g = oracle.lim03_grad([0.0, 0.0, 10.0], 1e-3)
    np.testing.assert_allclose(g, [0.0, 1.0, 0.0], atol=1e-12)


# --------------------------------------------------------------- whole scheme
def test_free_stream_and_conservation():
    with oracle.use_recon(oracle.LIM03):
        bs = inputs.orszag_tang_2d(32, 16)
        out, _ = oracle.run(bs, oracle.SSPRK43, 6)
        for v in range(bs.nvar):
            a, b = total(bs, v), total(out, v)
            assert abs(a - b) <= 1e-12 * max(1.0, abs(a)), v
        uni = inputs.density_wave_1d(32, amp=0.0)
        L, _ = oracle.rhs(uni)
        assert np.all(uni.interior(0, L[0]) == 0.0)
        out, _ = oracle.run(uni, oracle.RK3, 5)
        np.testing.assert_allclose(out.interior(0), uni.interior(0), rtol=1e-15)


def test_block_decomposition_is_bitwise_invisible():
    with oracle.use_recon(oracle.LIM03):
        one = inputs.orszag_tang_2d(32, 32)
        many = inputs.orszag_tang_2d(32, 8)
        a, dta = oracle.run(one, oracle.RK3, 4)
        b, dtb = oracle.run(many, oracle.RK3, 4)
    assert np.array_equal(dta, dtb)
    ua = a.interior(0)
    for blk in range(many.nb):
        ox = int(round((many.xlo[blk, 0] - one.xlo[0, 0]) / many.dx[blk, 0]))
        oy = int(round((many.xlo[blk, 1] - one.xlo[0, 1]) / many.dx[blk, 1]))
        sub = ua[:, :, oy:oy + 8, ox:ox + 8]
        assert np.array_equal(sub, b.interior(blk)), blk


def test_density_wave_third_order():
    errs = []
    with oracle.use_recon(oracle.LIM03):
        for N in (32, 64, 128):
            bs = inputs.density_wave_1d(N)
            dt, n = fixed_dt(bs, 0.5)
            out, _ = oracle.run(bs, oracle.RK3, n, dt=dt)
            x = (np.arange(N) + 0.5) / N
            rho = out.interior(0)[0].ravel()
            errs.append(np.abs(rho - (1 + 0.2 * np.sin(2 * math.pi * (x - 0.5)))).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.9 < o < 3.2 for o in orders), orders


def test_alfven_wave_third_order_in_both_norms():
    order = paper_number("alfven_observed_order_lim03_rk3")
    l1, linf = [], []
    with oracle.use_recon(oracle.LIM03):
        for N in (16, 32, 64):
            bs = inputs.circular_alfven(1, N)
            dt, n = fixed_dt(bs, 1.0)
            out, _ = oracle.run(bs, oracle.RK3, n, dt=dt)
            d = np.abs(out.interior(0) - bs.interior(0))
            l1.append(d.mean(axis=(1, 2, 3)))
            linf.append(d.max(axis=(1, 2, 3)))
    l1, linf = np.array(l1), np.array(linf)
    for v in (2, 3, 6, 7):
        for E in (l1, linf):
            o = np.log2(E[:-1, v] / E[1:, v])
            assert np.all(o > order - 0.2), (v, o)


def test_brio_wu_contact_without_overshoot():
    N = int(paper_number("brio_wu_cells"))
    t_end = paper_number("brio_wu_t_end")
    cfl = paper_number("brio_wu_courant")

    def overshoot(recon, scheme):
        with oracle.use_recon(recon):
            out = run_to_time(inputs.brio_wu(N), t_end, cfl=cfl, scheme=scheme)
        x = out.xlo[0, 0] + (np.arange(N) + 0.5) * out.dx[0, 0]
        rho = out.interior(0)[0].ravel()
        idx = np.where((x > 0.0) & (x < 0.25))[0]
        xc = x[idx[np.argmin(np.diff(rho[idx]))]]
        plateau = np.median(rho[(x > xc - 0.12) & (x < xc - 0.03)])
        peak = rho[(x > xc - 0.03) & (x <= xc)].max()
        return 100 * (peak / plateau - 1)

    lim = overshoot(oracle.LIM03, oracle.RK3)
    mp5 = overshoot(oracle.MP5, oracle.SSPRK54)
    assert abs(lim - paper_number("brio_wu_lim03_fd_density_overshoot_percent")) < 1.0, lim
    assert mp5 - lim > 1.5, (mp5, lim)


def test_brio_wu_at_the_maximal_ssp_courant_numbers():
    # Sect. 4.5.2: both FD combinations run the tube at the largest Courant
    # number their SSP property allows; MP5's oscillation level there is
    # comparable to Courant 0.4, while the third-order scheme departs more.
    N = int(paper_number("brio_wu_cells"))
    t_end = paper_number("brio_wu_t_end")

    def vy(recon, scheme, cfl):
        with oracle.use_recon(recon):
            out = run_to_time(inputs.brio_wu(N), t_end, cfl=cfl, scheme=scheme)
        u = out.interior(0)[:, 0, 0, :]
        rho, E = u[0], u[4]
        p = (paper_number("brio_wu_gamma") - 1) * (E - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / rho
                                                   - 0.5 * (u[5] ** 2 + u[6] ** 2 + u[7] ** 2))
        assert np.all(rho > 0) and np.all(p > 0)
        return u[2] / rho

    lim_lo = vy(oracle.LIM03, oracle.SSPRK43, 0.4)
    lim_hi = vy(oracle.LIM03, oracle.SSPRK43, paper_number("brio_wu_ssp_courant_ssprk43_lim03"))
    mp5_lo = vy(oracle.MP5, oracle.SSPRK54, 0.4)
    mp5_hi = vy(oracle.MP5, oracle.SSPRK54, paper_number("brio_wu_ssp_courant_ssprk54_mp5"))
    tv = lambda a: np.abs(np.diff(a)).sum()
    assert abs(tv(mp5_hi) / tv(mp5_lo) - 1.0) < 0.05
    assert np.abs(lim_hi - lim_lo).max() > 2.0 * np.abs(mp5_hi - mp5_lo).max()
