"""Pins of the oracle's MP5 reconstruction (Suresh & Huynh 1997, selected in
Sect. 2.2): exactness on polynomials, monotonicity preservation, accuracy at
smooth extrema, symmetries, and the derivative of the branch taken."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs


def cell_average(coeffs, a, b):
    """Exact mean of the polynomial sum c_k x^k over [a, b]."""
    P = np.polynomial.polynomial.polyint(coeffs)
    return (np.polynomial.polynomial.polyval(b, P) - np.polynomial.polynomial.polyval(a, P)) / (b - a)


@pytest.mark.parametrize("seed", range(8))
def test_reconstruction_exact_for_quartic_cell_averages(seed):
    # Monotone quartic: the limiter stays inactive and the 5-cell stencil
    # reproduces the interface value of a degree <= 4 polynomial exactly.
    rng = np.random.default_rng(seed)
    h = 0.05
    c = np.array([0.3, 1.0, rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)])
    x0 = rng.uniform(-0.2, 0.2)
    f = [cell_average(c, x0 + (j - 0.5) * h, x0 + (j + 0.5) * h) for j in (-2, -1, 0, 1, 2)]
    exact = np.polynomial.polynomial.polyval(x0 + 0.5 * h, c)
    assert abs(oracle.mp5(f) - exact) < 1e-13


@pytest.mark.parametrize("seed", range(8))
def test_fd_derivative_exact_for_quintic_point_values(seed):
    # Conservative FD derivative (Sect. 2.1): (Fhat_{i+1/2} - Fhat_{i-1/2})/dx
    # equals g'(x_i) exactly for point values of a polynomial of degree <= 5.
    rng = np.random.default_rng(100 + seed)
    h = 0.02
    c = np.array([0.1, 1.0, *rng.uniform(-0.4, 0.4, size=4)])
    xi = rng.uniform(-0.3, 0.3)
    pts = [np.polynomial.polynomial.polyval(xi + j * h, c) for j in range(-3, 3)]
    right = oracle.mp5(pts[1:6])   # interface i+1/2 from f_{i-2..i+2}
    left = oracle.mp5(pts[0:5])    # interface i-1/2 from f_{i-3..i+1}
    deriv = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(c))
    assert abs((right - left) / h - deriv) < 1e-10 * max(1.0, abs(deriv))


def test_degree6_converges_at_fifth_order():
    errs = []
    for h in (0.04, 0.02, 0.01):
        c = np.array([0.0, 1.0, 0.2, 0.1, 0.05, 0.02, 0.3])
        pts = [np.polynomial.polynomial.polyval(j * h, c) for j in range(-3, 3)]
        d = (oracle.mp5(pts[1:6]) - oracle.mp5(pts[0:5])) / h
        errs.append(abs(d - np.polynomial.polynomial.polyval(0.0, np.polynomial.polynomial.polyder(c))))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(4.8 < o < 5.2 for o in orders), orders


def test_monotone_data_stays_between_centre_and_neighbour():
    rng = np.random.default_rng(7)
    for _ in range(20000):
        f = np.sort(rng.normal(size=5)) * rng.choice([-1.0, 1.0])
        r = oracle.mp5(f)
        assert min(f[2], f[3]) <= r <= max(f[2], f[3])


def test_step_produces_no_overshoot():
    for f in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [1, 1, 1, 0, 0], [0, 0, 0, 0, 1], [0, 1, 1, 1, 1]):
        r = oracle.mp5(np.array(f, float))
        assert 0.0 <= r <= 1.0


def test_isolated_spike_is_not_amplified():
    r = oracle.mp5([0.0, 0.0, 1.0, 0.0, 0.0])
    assert 0.0 <= r <= 1.0
    r = oracle.mp5([0.0, 1.0, 0.0, 1.0, 0.0])
    assert 0.0 <= r <= 1.0


def test_smooth_extremum_keeps_high_order():
    # At a smooth maximum a plain minmod/TVD limiter clips to the centre value;
    # MP5's curvature-based bounds keep the interface value accurate.
    errs = []
    for h in (0.1, 0.05, 0.025):
        pts = [math.cos(j * h) for j in range(-3, 3)]
        d = (oracle.mp5(pts[1:6]) - oracle.mp5(pts[0:5])) / h
        errs.append(abs(d - 0.0))   # g'(0) = 0 at the maximum
    assert errs[-1] < 1e-6
    assert math.log2(errs[0] / errs[1]) > 3.5 or errs[1] < 1e-12
    # one-sided value next to the peak is close to the exact interface value
    h = 0.05
    pts = [math.cos((j - 0.5) * h) for j in range(-2, 3)]   # peak between j=0 and j=1 (shifted)
    assert abs(oracle.mp5(pts) - 1.0) < 1e-3


@pytest.mark.parametrize("seed", range(4))
def test_odd_symmetry_and_power_of_two_scaling_bitwise(seed):
    rng = np.random.default_rng(seed)
    for _ in range(2000):
        f = rng.normal(size=5)
        r = oracle.mp5(f)
        assert oracle.mp5(-f) == -r
        assert oracle.mp5(4.0 * f) == 4.0 * r
        assert oracle.mp5(0.125 * f) == 0.125 * r


def test_affine_equivariance():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        f = rng.normal(size=5)
        s = rng.uniform(0.1, 10.0)
        t = rng.normal()
        assert abs(oracle.mp5(s * f + t) - (s * oracle.mp5(f) + t)) < 1e-12 * (1 + abs(t) + s)


def test_constant_data():
    for v in (0.0, 0.5, -3.25, 2.5):
        assert oracle.mp5([v] * 5) == v


def test_gradient_of_branch_taken_matches_differences():
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(3000):
        f = rng.normal(size=5)
        v, g = oracle.mp5_grad(f)
        assert v == oracle.mp5(f)
        h = 1e-7
        fd = np.zeros(5)
        for i in range(5):
            e = np.zeros(5); e[i] = h
            fd[i] = (oracle.mp5(f + e) - oracle.mp5(f - e)) / (2 * h)
        # piecewise linear: away from kinks the central difference is exact
        if np.max(np.abs(fd - g)) < 1e-6:
            checked += 1
    assert checked > 2900   # kinks are met only on a set of small measure


def test_unlimited_gradient_is_the_linear_formula():
    _, g = oracle.mp5_grad([1.0, 2.0, 3.0, 4.0, 5.0])
    np.testing.assert_allclose(g * 60.0, [2, -13, 47, 27, -3], atol=1e-12)
    assert abs(g.sum() - 1.0) < 1e-15


def test_median_form_equals_the_early_exit_bitwise():
    """With eps = 0 the early exit returns a value inside both bounds, so
    MP5 without it (the median form, an option of the oracle's operation
    counter) gives the same bits: random tuples, monotone runs, extrema,
    flat stencils and one-sided kinks."""
    rng = np.random.default_rng(5)
    cases = [rng.normal(size=5) for _ in range(20000)]
    cases += [np.sort(rng.normal(size=5)) for _ in range(2000)]
    cases += [np.array([0.0, 1.0, 2.0, 1.0, 0.0]), np.full(5, 0.7), np.array([1.0, 1.0, 1.0, 2.0, 3.0]),
              np.array([0.0, 0.0, 1.0, 1.0, 1.0]), np.array([3.0, 1.0, 0.0, 1.0, 3.0])]
    ref = [oracle.mp5(f) for f in cases]
    with oracle.mp5_median_form():
        got = [oracle.mp5(f) for f in cases]
    assert got == ref


def test_operation_counter_units_and_a_hand_count():
    """orc_count_ops: the units match the loops of one SSPRK(5,4) step, and
    one hydro 1D flux unit (primitive recovery 6, flux 4, split 3 x 2 x 3)
    costs 28 arithmetic operations."""
    bs = inputs.density_wave_1d(64, nblocks=2)
    c = oracle.count_ops(bs, oracle.SSPRK54)
    st = 5
    assert c["flux"]["units"] == st * 2 * (32 + 6)
    assert c["recon"]["units"] == st * 2 * 2 * 3 * 33
    assert c["diff"]["units"] == st * 2 * 3 * 32
    assert c["stage"]["units"] == st * 64
    assert c["cmax"]["units"] == st * 64
    assert c["flux"]["ops"] == 28 * c["flux"]["units"]
    assert c["flux"]["cmp"] == 0
    # the median form costs more arithmetic per reconstruction
    m = oracle.count_ops(bs, oracle.SSPRK54, median_form=True)
    assert m["recon"]["ops"] > c["recon"]["ops"]
    assert m["flux"]["ops"] == c["flux"]["ops"]
