"""Pins of the oracle's physics: primitive recovery against the input
generator's (independent) prim->cons map, fluxes against their
characteristic speeds (eigenvalues of the numerical flux Jacobian), and the
closed-form limits of the fast speed."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs


def cons(ndim, mhd, gamma, **w):
    one = np.ones((1, 1, 1))
    fields = {k: v * one for k, v in w.items()}
    return inputs.conserved_from_prims(ndim, mhd, gamma, fields)[:, 0, 0, 0]


def random_prims(rng, mhd):
    w = {"rho": rng.uniform(0.5, 2.0), "p": rng.uniform(0.2, 2.0),
         "vx": rng.normal(), "vy": rng.normal(), "vz": rng.normal()}
    if mhd:
        w.update({"Bx": rng.normal(), "By": rng.normal(), "Bz": rng.normal()})
    return w


@pytest.mark.parametrize("ndim,mhd", [(1, False), (2, False), (3, False), (1, True), (3, True)])
def test_prim_roundtrip(ndim, mhd):
    rng = np.random.default_rng(ndim + 10 * mhd)
    for _ in range(200):
        w = random_prims(rng, mhd)
        u = cons(ndim, mhd, 1.4, **w)
        st, got = oracle.prim(ndim, mhd, 1.4, u)
        assert st == 0
        exp = [w["rho"], w["vx"], w["vy"] if (mhd or ndim > 1) else 0.0,
               w["vz"] if (mhd or ndim > 2) else 0.0, w["p"]]
        np.testing.assert_allclose(got[:5], exp, rtol=1e-12, atol=1e-12)


def test_nonphysical_states_are_rejected():
    st, _ = oracle.prim(1, False, 1.4, [-1.0, 0.0, 1.0])
    assert st == 4
    st, _ = oracle.prim(1, False, 1.4, [1.0, 2.0, 1.0])   # E < kinetic -> p < 0
    assert st == 4
    st, _ = oracle.prim(1, False, 1.4, [1.0, float("nan"), 1.0])
    assert st == 4


def jac_eigs(ndim, mhd, gamma, d, u):
    n = len(u)
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * max(1.0, abs(u[j]))
        e = np.zeros(n); e[j] = h
        J[:, j] = (oracle.flux(ndim, mhd, gamma, d, u + e) - oracle.flux(ndim, mhd, gamma, d, u - e)) / (2 * h)
    return np.sort(np.linalg.eigvals(J).real)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_hydro_flux_characteristic_speeds(ndim):
    rng = np.random.default_rng(ndim)
    g = 1.4
    for _ in range(20):
        w = random_prims(rng, False)
        u = cons(ndim, False, g, **w)
        for d in range(ndim):
            v = [w["vx"], w["vy"], w["vz"]][d]
            cs = math.sqrt(g * w["p"] / w["rho"])
            ev = jac_eigs(ndim, False, g, d, u)
            exp = np.sort([v - cs] + [v] * ndim + [v + cs])
            np.testing.assert_allclose(ev, exp, atol=2e-6)
            assert abs(oracle.fast_speed(ndim, False, g, d, u) - cs) < 1e-14


@pytest.mark.parametrize("d", [0, 1, 2])
def test_mhd_flux_characteristic_speeds(d):
    # The 8x8 Jacobian of the ideal MHD flux along d has the seven MHD waves
    # v-cf, v-ca, v-cs, v, v+cs, v+ca, v+cf plus 0 (the normal-field row is
    # identically zero).  The fast speed of the oracle must equal the
    # largest |eigenvalue - v|.
    rng = np.random.default_rng(50 + d)
    g = 5.0 / 3.0
    for _ in range(20):
        w = random_prims(rng, True)
        u = cons(3, True, g, **w)
        ev = jac_eigs(3, True, g, d, u)
        # drop the zero eigenvalue of the identically-zero normal-field flux
        ev = np.delete(ev, np.argmin(np.abs(ev)))
        v = [w["vx"], w["vy"], w["vz"]][d]
        cf = oracle.fast_speed(3, True, g, d, u)
        assert abs(ev.max() - (v + cf)) < 1e-5
        assert abs(ev.min() - (v - cf)) < 1e-5
        B = np.array([w["Bx"], w["By"], w["Bz"]])
        ca = abs(B[d]) / math.sqrt(w["rho"])
        for s in (+1, -1):
            assert np.min(np.abs(ev - (v + s * ca))) < 1e-5
        assert np.min(np.abs(ev - v)) < 1e-5   # entropy wave


def test_fast_speed_limits():
    g = 5.0 / 3.0
    rho, p = 1.3, 0.7
    cs = math.sqrt(g * p / rho)
    # B = 0: sound speed
    u = cons(3, True, g, rho=rho, p=p, vx=0.1, vy=0.2, vz=0.3)
    for d in range(3):
        assert abs(oracle.fast_speed(3, True, g, d, u) - cs) < 1e-14
    # B parallel to d: max(cs, vA)
    for Bmag in (0.3, 2.0):
        u = cons(3, True, g, rho=rho, p=p, Bx=Bmag)
        vA = Bmag / math.sqrt(rho)
        assert abs(oracle.fast_speed(3, True, g, 0, u) - max(cs, vA)) < 1e-14
        # perpendicular: sqrt(cs^2 + vA^2)
        assert abs(oracle.fast_speed(3, True, g, 1, u) - math.sqrt(cs * cs + vA * vA)) < 1e-14


def test_mhd_flux_reduces_to_hydro_for_zero_field():
    g = 1.4
    rng = np.random.default_rng(9)
    for _ in range(50):
        w = random_prims(rng, False)
        uh = cons(3, False, g, **w)
        um = cons(3, True, g, **w)
        for d in range(3):
            fh = oracle.flux(3, False, g, d, uh)
            fm = oracle.flux(3, True, g, d, um)
            np.testing.assert_allclose(fm[:5], fh, rtol=1e-14, atol=1e-14)
            assert np.all(fm[5:] == 0.0)


def test_flux_rotation_covariance():
    # Flux along y of a state equals the flux along x of the state with x and
    # y exchanged (components permuted), for hydro and MHD.
    g = 5.0 / 3.0
    rng = np.random.default_rng(21)
    perm_h = [0, 2, 1, 3, 4]
    perm_m = [0, 2, 1, 3, 4, 6, 5, 7]
    for mhd, perm in ((False, perm_h), (True, perm_m)):
        for _ in range(30):
            w = random_prims(rng, mhd)
            u = cons(3, mhd, g, **w)
            uy = u[perm]
            fy = oracle.flux(3, mhd, g, 1, u)
            fx = oracle.flux(3, mhd, g, 0, uy)
            np.testing.assert_allclose(fy, fx[perm], rtol=1e-14, atol=1e-14)
