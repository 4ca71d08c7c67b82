"""Pins of the oracle's Hall MHD (Sect. 4.4, conservative Hall MHD in finite
differences: cell-centred current by fourth-order central differences, Hall
terms in the fluxes of B and E, whistler-augmented speeds): the flux terms
against the Hall electric field, the exact circularly polarised
Alfven-whistler waves of both branches in 1D and on an oblique 2D grid
(Sect. 4.5.3), the speeds, conservation and the refusal of fixed faces."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs
from test_oracle_solutions import fixed_dt, total

GAMMA = 5.0 / 3.0


@pytest.fixture(autouse=True)
def ideal_after():
    yield
    oracle.set_hall(0.0)


def test_flux_terms_are_the_hall_electric_field():
    # E_H = (eta_h/rho) J x B: the Hall part of the flux of B_k along d is
    # -eps_dkl E_l and that of the energy is (E_H x B)_d
    rng = np.random.default_rng(4)
    eps = np.zeros((3, 3, 3))
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        eps[a, b, c], eps[a, c, b] = 1.0, -1.0
    for _ in range(50):
        w = {"rho": np.array([1 + rng.uniform()]), "p": np.array([1 + rng.uniform()])}
        for key in ("vx", "vy", "vz", "Bx", "By", "Bz"):
            w[key] = np.array([rng.normal()])
        u = inputs.conserved_from_prims(3, True, GAMMA, w)[:, 0]
        J = rng.normal(size=3)
        eta = rng.uniform(0.1, 2.0)
        B = u[5:8]
        E = eta / u[0] * np.cross(J, B)
        for d in range(3):
            hall = oracle.flux_hall(3, GAMMA, eta, d, u, J) - oracle.flux(3, True, GAMMA, d, u)
            np.testing.assert_allclose(hall[5:8], [-np.dot(eps[d, k], E) for k in range(3)], atol=1e-13)
            assert hall[4] == pytest.approx(np.cross(E, B)[d], abs=1e-13)
            assert np.all(hall[:4] == 0.0)


def whistler_errors(ndim, Ns, d, branch, kvec=(1, 0, 0), scheme=oracle.SSPRK54):
    errs = []
    for N in Ns:
        bs, v, T = inputs.alfven_whistler(ndim, N, d, branch, kvec=kvec, block=N // 2)
        with oracle.use_hall(d):
            dt, n = fixed_dt(bs, T)
            out, _ = oracle.run(bs, scheme, n, dt=dt)
        errs.append(np.mean([np.abs(out.interior(b) - bs.interior(b)).mean() for b in range(bs.nb)]))
    return errs


@pytest.mark.parametrize("branch", [+1, -1], ids=["ion_cyclotron", "whistler"])
def test_alfven_whistler_wave_1d_fourth_order(branch):
    # one period of the exact wave: the error falls at fourth order (the
    # current's central differences) and is far below the amplitude
    errs = whistler_errors(1, (32, 64, 128), 0.2, branch)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.8 < o < 4.3 for o in orders), (errs, orders)
    assert errs[-1] < 1e-6


def test_hall_term_moves_the_wave():
    # the same state run as ideal MHD is far from the Hall solution
    bs, v, T = inputs.alfven_whistler(1, 64, 0.2, -1, block=32)
    dt, n = fixed_dt(bs, T)
    out, _ = oracle.run(bs, oracle.SSPRK54, n, dt=dt)
    assert np.mean([np.abs(out.interior(b) - bs.interior(b)).mean() for b in range(bs.nb)]) > 1e-2


def test_alfven_whistler_wave_oblique_2d():
    # k = 2 pi (1, 1): every component of curl B has cross-direction terms
    errs = whistler_errors(2, (16, 32), 0.1, -1, kvec=(1, 1, 0))
    assert math.log2(errs[0] / errs[1]) > 3.6, errs
    assert errs[-1] < 1e-5


def test_speeds_include_the_whistler_at_k_max():
    bs, v, T = inputs.alfven_whistler(2, 16, 0.3, -1, kvec=(1, 1, 0), block=8)
    ideal = oracle.cmax(bs)
    with oracle.use_hall(0.3):
        cm = oracle.cmax(bs)
    kmax = math.pi / bs.dx[0, 0]
    bmax = max(float(np.sqrt((bs.interior(b)[5:8] ** 2).sum(axis=0)).max()) for b in range(bs.nb))
    vmax = max(float(np.abs(bs.interior(b)[1:3]).max()) for b in range(bs.nb))
    for d in range(2):
        assert cm[d] > ideal[d]
        assert 0.3 * 0.9 * bmax * kmax < cm[d] <= 0.3 * bmax * kmax + vmax + 1e-12


def test_conservation_and_fixed_faces_refused():
    bs = inputs.orszag_tang_2d(32, 16)
    with oracle.use_hall(0.05):
        out, _ = oracle.run(bs, oracle.SSPRK54, 4)
        for v in range(8):
            a, b = total(bs, v), total(out, v)
            assert abs(a - b) <= 1e-12 * max(1.0, abs(a)), v
        with pytest.raises(oracle.OracleError):
            oracle.rhs(inputs.brio_wu(64))
