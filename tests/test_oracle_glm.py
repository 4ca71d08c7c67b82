"""Pins of the oracle's GLM-MHD (Sect. 4.2, the glm3 variant: psi as a ninth
variable with flux psi on B_d and c_h^2 B_d on psi, operator-split decay of
psi): reduction to ideal MHD, the +-c_h waves of the psi-B_n subsystem, the
exact decay of a uniform psi, conservation, and the paper's statement that
the divergence of B then falls with the order of the reconstruction minus
one (Sect. 4.5.1)."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs
from test_oracle_solutions import fixed_dt, total

GAMMA = 5.0 / 3.0


@pytest.fixture(autouse=True)
def glm_cr_default():
    yield
    oracle.set_glm_cr(0.18)


def test_flux_terms():
    # psi enters the flux of B_d only, c_h^2 B_d is the flux of psi, and
    # nothing else changes (glm3 has no other psi terms)
    rng = np.random.default_rng(1)
    for _ in range(50):
        w = {"rho": 1 + rng.uniform(), "p": 1 + rng.uniform(), "vx": rng.normal(), "vy": rng.normal(),
             "vz": rng.normal(), "Bx": rng.normal(), "By": rng.normal(), "Bz": rng.normal(), "psi": rng.normal()}
        u9 = inputs.conserved_from_prims(3, 2, GAMMA, {k: np.array([v]) for k, v in w.items()})[:, 0]
        ch = rng.uniform(0.5, 3.0)
        for d in range(3):
            f9 = oracle.flux_glm(3, GAMMA, d, ch, u9)
            f8 = oracle.flux(3, True, GAMMA, d, u9[:8])
            expect = f8.copy()
            expect[5 + d] += u9[8]
            np.testing.assert_allclose(f9[:8], expect, rtol=1e-14, atol=1e-14)
            assert f9[8] == pytest.approx(ch * ch * u9[5 + d], rel=1e-15)


def test_uniform_normal_field_in_1d_is_ideal_mhd_bitwise():
    # 1D with B_x constant: psi is never generated, c_h equals c_max,x, and
    # every operation on the other eight variables is the MHD one.
    mhd = inputs.brio_wu(128)
    glm = inputs.as_glm(mhd)
    a, dta = oracle.run(mhd, oracle.SSPRK54, 30)
    b, dtb = oracle.run(glm, oracle.SSPRK54, 30)
    assert np.array_equal(dta, dtb)
    assert np.array_equal(a.u[0], b.u[0][:8])
    assert np.all(b.u[0][8] == 0.0)


def psi_wave_state(N, eps, psi0=0.0):
    # B_x = eps b(x) with B_0 = 0, v = 0, uniform rho and p: to O(eps^2) the
    # (B_x, psi) pair obeys dB/dt + dpsi/dx = 0, dpsi/dt + c_h^2 dB/dx = 0
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(1, [N], [N // 4])
    return inputs.sample_blocks(1, 2, GAMMA, n, dx, xlo, nbr, lambda X, Y, Z: {
        "rho": 1.0 + 0 * X, "p": 1.0 + 0 * X, "Bx": eps * np.exp(-((X - 0.5) / 0.06) ** 2),
        "psi": psi0 + 0 * X})


def test_divergence_error_splits_into_two_waves_at_the_cleaning_speed():
    oracle.set_glm_cr(1e300)          # no decay: the pure hyperbolic subsystem
    N, eps, T = 256, 1e-6, 0.15
    bs = psi_wave_state(N, eps)
    c = oracle.cmax(bs)[0]            # = c_h (sound speed up to O(eps^2))
    assert c == pytest.approx(math.sqrt(GAMMA), rel=1e-9)
    dt, nsteps = fixed_dt(bs, T)
    out, _ = oracle.run(bs, oracle.SSPRK54, nsteps, dt=dt)
    x = (np.arange(N) + 0.5) / N
    b = lambda s: eps * np.exp(-((((s - 0.5) + 0.5) % 1.0 - 0.5) / 0.06) ** 2)
    Bx = np.concatenate([out.interior(i)[5].ravel() for i in range(out.nb)])
    psi = np.concatenate([out.interior(i)[8].ravel() for i in range(out.nb)])
    Bx_ex = 0.5 * (b(x - c * T) + b(x + c * T))
    psi_ex = 0.5 * c * (b(x - c * T) - b(x + c * T))
    assert np.abs(Bx - Bx_ex).max() < 2e-3 * eps
    assert np.abs(psi - psi_ex).max() < 2e-3 * eps * c
    # a sign error in either coupling would move the pulses the wrong way
    assert np.abs(psi + psi_ex).max() > 0.5 * eps


def test_uniform_psi_decays_exactly():
    # uniform psi, uniform B_x: fluxes are constant, only the operator-split
    # decay acts: psi_n = psi_0 prod exp(-dt c_h / c_r)
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(2, [16, 16], [8, 8])
    bs = inputs.sample_blocks(2, 2, GAMMA, n, dx, xlo, nbr, lambda X, Y, Z: {
        "rho": 1.0 + 0 * X, "p": 0.5 + 0 * X, "vx": 0.3 + 0 * X, "Bx": 0.7 + 0 * X, "By": 0.2 + 0 * X,
        "psi": 0.25 + 0 * X})
    ch = oracle.cmax(bs).max()
    out, dts = oracle.run(bs, oracle.RK3, 7)
    expect = 0.25 * math.exp(-dts.sum() * ch / oracle.glm_cr())
    for b in range(out.nb):
        np.testing.assert_allclose(out.interior(b)[8], expect, rtol=1e-13)
        np.testing.assert_allclose(out.interior(b)[:8], bs.interior(b)[:8], rtol=1e-14, atol=1e-15)


def test_every_direction_uses_the_cleaning_speed():
    # 2D: c_max,d <- c_h = max_d c_max,d in the split and in the time step
    bs = inputs.as_glm(inputs.orszag_tang_2d(32, 16))
    cm = oracle.cmax(bs)
    cm_mhd = oracle.cmax(inputs.orszag_tang_2d(32, 16))
    assert cm[0] == cm[1] == max(cm_mhd[0], cm_mhd[1])
    _, dts = oracle.run(bs, oracle.SSPRK54, 1)
    assert dts[0] == pytest.approx(0.4 / (cm[0] / bs.dx[0, 0] + cm[1] / bs.dx[0, 1]), rel=1e-15)


def test_conservation_and_psi_budget():
    bs = inputs.as_glm(inputs.orszag_tang_2d(32, 8), psi=0.0)
    out, dts = oracle.run(bs, oracle.SSPRK54, 5)
    for v in range(8):
        a, b = total(bs, v), total(out, v)
        assert abs(a - b) <= 1e-12 * max(1.0, abs(a)), v
    # psi is generated by the discrete divergence of B and stays finite
    assert np.isfinite(total(out, 8))


def divb_mean(out):
    """Mean |div B| of a 2D periodic unit-square list by fourth-order central
    differences on the assembled global array."""
    N = int(round(1.0 / out.dx[0, 0]))
    h = 1.0 / N
    g = np.zeros((3, N, N))
    for b in range(out.nb):
        ox = int(round(out.xlo[b, 0] / h)); oy = int(round(out.xlo[b, 1] / h))
        g[:, oy:oy + out.n[b, 1], ox:ox + out.n[b, 0]] = out.interior(b)[5:8, 0]
    d4 = lambda f, ax: (8 * (np.roll(f, -1, ax) - np.roll(f, 1, ax))
                        - (np.roll(f, -2, ax) - np.roll(f, 2, ax))) / (12 * h)
    return np.abs(d4(g[0], 1) + d4(g[1], 0)).mean()


def test_divergence_falls_with_reconstruction_order_minus_one():
    # Sect. 4.5.1: with GLM the divergence of B decreases with the order of
    # the reconstruction minus one: fourth order with MP5.  An oblique wave
    # (k = 2 pi (1, 2)) so that the grid directions see different stencil
    # errors (along the diagonal div B stays at rounding by symmetry).
    errs = []
    for N in (16, 32, 64):
        bs = inputs.circular_alfven(2, N, block=N // 2, kvec=(1, 2, 0), glm=True)
        T = 1.0 / math.sqrt(5.0)
        dt, n = fixed_dt(bs, T)
        out, _ = oracle.run(bs, oracle.SSPRK54, n, dt=dt)
        errs.append(divb_mean(out))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(o > 3.5 for o in orders), (errs, orders)


def test_glm_alfven_wave_fifth_order():
    E = []
    for N in (16, 32):
        bs = inputs.circular_alfven(2, N, block=N // 2, kvec=(1, 1, 0), glm=True)
        T = 1.0 / math.sqrt(2.0)
        dt, n = fixed_dt(bs, T)
        out, _ = oracle.run(bs, oracle.SSPRK54, n, dt=dt)
        E.append(np.mean([np.abs(out.interior(b)[:8] - bs.interior(b)[:8]).mean(axis=(1, 2, 3))
                          for b in range(bs.nb)], axis=0))
    E = np.array(E)
    for v in (2, 6, 7):
        assert math.log2(E[0, v] / E[1, v]) > 4.5, (v, E[:, v])


# --------------------------------------------------------------- div B monitor
def test_divb_exact_for_quartic_fields_with_fixed_ghosts():
    # fourth-order central differences are exact for polynomials of degree <= 4
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(3, [12, 10, 8], [6, 5, 8], periodic=False)
    f = lambda X, Y, Z: {"rho": 1.0 + 0 * X, "p": 1.0 + 0 * X, "Bx": X ** 4 - 2 * X * Y + Z,
                         "By": Y ** 3 * Z + X ** 2, "Bz": Z ** 2 * X - Y}
    bs = inputs.sample_blocks(3, True, GAMMA, n, dx, xlo, nbr, f)
    div = oracle.divb(bs)
    for b in range(bs.nb):
        X, Y, Z = inputs.cell_centres(3, bs.n[b], bs.dx[b], bs.xlo[b])
        exact = 4 * X ** 3 - 2 * Y + 3 * Y ** 2 * Z + 2 * Z * X
        np.testing.assert_allclose(div[b], exact[3:-3, 3:-3, 3:-3], rtol=0, atol=1e-11)


def test_divb_zero_for_fields_constant_along_their_own_direction():
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(3, [16, 16, 16], [8, 8, 8])
    tp = 2 * math.pi
    bs = inputs.sample_blocks(3, 2, GAMMA, n, dx, xlo, nbr, lambda X, Y, Z: {
        "rho": 1.0 + 0 * X, "p": 1.0 + 0 * X, "Bx": np.sin(tp * Y) + np.cos(tp * Z),
        "By": np.sin(tp * Z) * np.cos(tp * X), "Bz": np.sin(tp * X + tp * Y)})
    for d in oracle.divb(bs):
        assert np.all(d == 0.0)


def test_divb_fourth_order_and_block_invariance():
    tp = 2 * math.pi
    errs = []
    for N in (16, 32, 64):
        n, dx, xlo, nbr, _ = inputs.uniform_blocks(2, [N, N], [N // 4, N // 2])
        bs = inputs.sample_blocks(2, True, GAMMA, n, dx, xlo, nbr, lambda X, Y, Z: {
            "rho": 1.0 + 0 * X, "p": 1.0 + 0 * X, "Bx": np.sin(tp * X), "By": np.cos(tp * Y)})
        div = oracle.divb(bs)
        err = 0.0
        for b in range(bs.nb):
            X, Y, Z = inputs.cell_centres(2, bs.n[b], bs.dx[b], bs.xlo[b])
            exact = (tp * np.cos(tp * X) - tp * np.sin(tp * Y))[:, 3:-3, 3:-3]
            err = max(err, np.abs(div[b] - exact).max())
        errs.append(err)
        one = inputs.sample_blocks(2, True, GAMMA, *inputs.uniform_blocks(2, [N, N], [N, N])[:4],
                                   lambda X, Y, Z: {"rho": 1.0 + 0 * X, "p": 1.0 + 0 * X,
                                                    "Bx": np.sin(tp * X), "By": np.cos(tp * Y)})
        whole = oracle.divb(one)[0]
        for b in range(bs.nb):
            ox = int(round(bs.xlo[b, 0] * N)); oy = int(round(bs.xlo[b, 1] * N))
            assert np.array_equal(div[b], whole[:, oy:oy + bs.n[b, 1], ox:ox + bs.n[b, 0]])
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.9 < o < 4.1 for o in orders), orders
