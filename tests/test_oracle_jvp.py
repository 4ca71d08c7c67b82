"""Pins of the oracle's forward-mode JVP of the time integration (used to
check the hand-written adjoint): central differences of the forward map,
linearity, and the c_max (argmax) term."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs


def axpy(bs, a, t):
    out = bs.copy()
    out.u = [u + a * x for u, x in zip(bs.u, t)]
    return out


def dot(a, b):
    return math.fsum(float(np.vdot(x, y)) for x, y in zip(a, b))


def smooth_hydro_2d(N=16, block=8):
    """2D Euler state with no flat field (every split flux varies in space)
    and no symmetry that would tie the c_max candidates of two cells."""
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(2, [N, N], [block, block])
    tp = 2 * math.pi
    return inputs.sample_blocks(2, False, 1.4, n, dx, xlo, nbr, lambda X, Y, Z: {
        "rho": 1 + 0.1 * np.sin(tp * X + 0.3) * np.sin(tp * Y + 0.7) + 0.03 * np.cos(tp * (X - 2 * Y) + 0.1),
        "vx": 0.5 + 0.1 * np.cos(tp * Y + 0.2), "vy": 0.3 + 0.1 * np.sin(tp * X + 1.1),
        "p": 1 + 0.1 * np.cos(tp * (X + Y) + 0.4)})


def random_mhd(ndim, N, block, seed):
    """MHD state built from seeded random-phase modes: no flat field and no
    symmetry tying the c_max candidates of two cells."""
    rng = np.random.default_rng(seed)
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(ndim, [N] * ndim, [block] * ndim)
    names = ["rho", "vx", "vy", "vz", "p", "Bx", "By", "Bz"]
    base = {"rho": 1.0, "vx": 0.2, "vy": -0.1, "vz": 0.05, "p": 1.0, "Bx": 0.8, "By": 0.3, "Bz": -0.2}
    modes = {k: [(rng.integers(1, 3, size=3), rng.uniform(0, 2 * math.pi)) for _ in range(2)]
             for k in names}

    def f(X, Y, Z):
        out = {}
        for k in names:
            acc = base[k]
            for kv, ph in modes[k]:
                acc = acc + 0.05 * np.sin(2 * math.pi * (kv[0] * X + kv[1] * Y + kv[2] * Z) + ph)
            out[k] = acc
        return out
    return inputs.sample_blocks(ndim, True, 5 / 3, n, dx, xlo, nbr, f)


@pytest.mark.parametrize("case", ["hydro2d", "hydro2d_rest_density", "mhd2d", "mhd1d",
                                  "lim03_hydro2d", "lim03_mhd2d", "lim03_limited_mhd1d"])
def test_jvp_matches_central_differences(case):
    # LIM03 cases: the default radius mixes the asymptotic and the limited
    # branches; a tiny radius sends every reconstruction through the
    # limited function.
    if case.startswith("lim03_limited_"):
        oracle.set_lim03_radius(1e-6)
        try:
            with oracle.use_recon(oracle.LIM03):
                return _jvp_case(case[14:], oracle.SSPRK43)
        finally:
            oracle.set_lim03_radius(1.0)
    if case.startswith("lim03_"):
        with oracle.use_recon(oracle.LIM03):
            return _jvp_case(case[6:], oracle.RK3 if case.endswith("hydro2d") else oracle.SSPRK43)
    return _jvp_case(case, None)


def _jvp_case(case, scheme_override):
    # Central differences are exact only where the forward map is smooth
    # ("non-kinked"): a state at rest makes the momentum and energy split
    # fluxes exactly flat, a kink of MP5, so there only density directions
    # (which keep those fluxes flat) are differentiable.
    if case == "hydro2d":
        bs = smooth_hydro_2d()
        tang = inputs.random_tangent(bs, 7)
        scheme, nsteps = oracle.SSPRK54, 3
    elif case == "hydro2d_rest_density":
        bs = inputs.hydro_random_2d(16, 8, seed=2)
        tang = inputs.random_tangent(bs, 7, vars_=[0])
        scheme, nsteps = oracle.SSPRK54, 3
    elif case == "mhd2d":
        bs = random_mhd(2, 16, 8, seed=1)
        tang = inputs.random_tangent(bs, 8)
        scheme, nsteps = oracle.SSPRK54, 2
    else:
        bs = random_mhd(1, 32, 8, seed=2)
        tang = inputs.random_tangent(bs, 9)
        scheme, nsteps = oracle.RK3, 4
    if scheme_override is not None:
        scheme = scheme_override
    _, cm = oracle.rhs(bs)
    dt = 0.3 / sum(cm[d] / bs.dx[0, d] for d in range(bs.ndim))
    _, du = oracle.run_jvp(bs, tang, scheme, nsteps, dt)
    # largest step at which both runs take the same branches as U0
    h0 = oracle.run_branch_hash(bs, scheme, nsteps, dt)
    for h in (1e-6, 1e-7, 1e-8):
        if (oracle.run_branch_hash(axpy(bs, h, tang), scheme, nsteps, dt) == h0 and
                oracle.run_branch_hash(axpy(bs, -h, tang), scheme, nsteps, dt) == h0):
            break
    else:
        pytest.fail("no non-kinked step found")
    plus, _ = oracle.run(axpy(bs, h, tang), scheme, nsteps, dt=dt)
    minus, _ = oracle.run(axpy(bs, -h, tang), scheme, nsteps, dt=dt)
    for b in range(bs.nb):
        fd = (plus.interior(b) - minus.interior(b)) / (2 * h)
        an = bs.interior(b, du[b])
        scale = max(np.abs(an).max(), 1e-3)
        assert np.abs(fd - an).max() < 1e-6 * scale, (b, h, np.abs(fd - an).max(), scale)


def test_branch_hash_detects_an_argmax_switch():
    # at h = 1e-5 the rest-density case switches the c_max argmax (the
    # difference quotient is then wrong by O(1)); the fingerprint must see it
    bs = inputs.hydro_random_2d(16, 8, seed=2)
    tang = inputs.random_tangent(bs, 7, vars_=[0])
    _, cm = oracle.rhs(bs)
    dt = 0.3 / sum(cm[d] / bs.dx[0, d] for d in range(bs.ndim))
    h0 = oracle.run_branch_hash(bs, oracle.SSPRK54, 2, dt)
    assert oracle.run_branch_hash(bs, oracle.SSPRK54, 2, dt) == h0
    assert oracle.run_branch_hash(axpy(bs, 1e-5, tang), oracle.SSPRK54, 2, dt) != h0


def test_jvp_value_part_equals_forward_run():
    bs = inputs.orszag_tang_2d(16, 8)
    tang = inputs.random_tangent(bs, 1)
    _, cm = oracle.rhs(bs)
    dt = 0.3 / sum(cm[d] / bs.dx[0, d] for d in range(bs.ndim))
    val, _ = oracle.run_jvp(bs, tang, oracle.SSPRK54, 2, dt)
    ref, _ = oracle.run(bs, oracle.SSPRK54, 2, dt=dt)
    for b in range(bs.nb):
        assert np.array_equal(val.interior(b), ref.interior(b))


def test_jvp_is_linear_in_the_tangent():
    bs = inputs.hydro_random_2d(16, 8, seed=3)
    t1 = inputs.random_tangent(bs, 11)
    t2 = inputs.random_tangent(bs, 12)
    dt = 1e-3
    _, a = oracle.run_jvp(bs, t1, oracle.SSPRK54, 2, dt)
    _, b = oracle.run_jvp(bs, t2, oracle.SSPRK54, 2, dt)
    _, a2 = oracle.run_jvp(bs, [2.0 * x for x in t1], oracle.SSPRK54, 2, dt)
    _, s = oracle.run_jvp(bs, [x + y for x, y in zip(t1, t2)], oracle.SSPRK54, 2, dt)
    for i in range(bs.nb):
        assert np.array_equal(a2[i], 2.0 * a[i])
        np.testing.assert_allclose(s[i], a[i] + b[i], rtol=1e-12, atol=1e-13)


def test_cmax_derivative_reaches_the_maximising_cell():
    # Perturb only the cell that attains c_max: the global LF speed changes,
    # so the tangent spreads to every cell after one stage (the split uses
    # c_max everywhere), and it agrees with central differences.
    bs = inputs.hydro_random_2d(16, 8, seed=5)
    best, where = -1.0, None
    g = bs.gamma
    for b in range(bs.nb):
        rho, mx, my, E = bs.interior(b)
        p = (g - 1) * (E - 0.5 * (mx * mx + my * my) / rho)
        c = np.sqrt(g * p / rho) + np.abs(mx / rho)
        i = np.unravel_index(np.argmax(c), c.shape)
        if c[i] > best:
            best, where = c[i], (b, i)
    b0, (k, j, i) = where
    tang = [np.zeros_like(u) for u in bs.u]
    tang[b0][0, k, j + 3, i + 3] = 1.0
    dt = 1e-3
    _, du = oracle.run_jvp(bs, tang, oracle.SSPRK54, 1, dt)
    far = (b0 + bs.nb // 2) % bs.nb
    assert np.abs(bs.interior(far, du[far])).max() > 0.0
    h = 1e-7
    plus, _ = oracle.run(axpy(bs, h, tang), oracle.SSPRK54, 1, dt=dt)
    minus, _ = oracle.run(axpy(bs, -h, tang), oracle.SSPRK54, 1, dt=dt)
    fd = (plus.interior(far) - minus.interior(far)) / (2 * h)
    np.testing.assert_allclose(bs.interior(far, du[far]), fd, atol=1e-7)
