"""Pins of the oracle's SSPRK tables (Sect. 2.3) against the printed values and
against the Runge-Kutta order conditions, stability polynomials and SSP
coefficients they must satisfy."""
import math

import numpy as np
import pytest

import oracle
from conftest import golden


def read_golden():
    rows = {}
    with open(golden("ssprk_tables.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            sch, kind, i, k, val = line.split()
            rows.setdefault(sch, []).append((kind, i, k, float(val)))
    return rows


def butcher(alpha, beta):
    """Shu-Osher -> Butcher: U(i) = U^n + dt sum_j c(i)_j L(U(j))."""
    s = alpha.shape[1]
    C = np.zeros((s + 1, s))
    for i in range(1, s + 1):
        assert abs(alpha[i, :i].sum() - 1.0) < 1e-13
        for k in range(i):
            C[i] += alpha[i, k] * C[k]
            C[i, k] += beta[i, k]
    return C[:s], C[s]


def order_residuals(A, b):
    c = A.sum(axis=1)
    return {
        "b": b.sum() - 1.0,
        "bc": b @ c - 1.0 / 2,
        "bc2": b @ c**2 - 1.0 / 3,
        "bAc": b @ A @ c - 1.0 / 6,
        "bc3": b @ c**3 - 1.0 / 4,
        "bcAc": (b * c) @ A @ c - 1.0 / 8,
        "bAc2": b @ A @ c**2 - 1.0 / 12,
        "bAAc": b @ A @ A @ c - 1.0 / 24,
    }


def stability_poly(A, b):
    s = len(b)
    one = np.ones(s)
    coeffs = [1.0]
    v = one.copy()
    for _ in range(s):
        coeffs.append(b @ v)
        v = A @ v
    return np.array(coeffs)


@pytest.mark.parametrize("name,scheme", [("ssprk43", oracle.SSPRK43), ("ssprk54", oracle.SSPRK54)])
def test_tables_match_printed_values(name, scheme):
    s, al, be = oracle.scheme_table(scheme)
    for kind, i, k, val in read_golden()[name]:
        if kind == "ssp_cfl":
            continue
        got = (al if kind == "alpha" else be)[int(i), int(k)]
        # alpha_50 is renormalised so the row sums to 1 (a change below 1e-13)
        assert abs(got - val) <= 1e-13, (kind, i, k, got, val)
    # every coefficient not printed is zero
    printed = {(kind, int(i), int(k)) for kind, i, k, _ in read_golden()[name] if kind != "ssp_cfl"}
    for i in range(1, s + 1):
        for k in range(s):
            if ("alpha", i, k) not in printed:
                assert al[i, k] == 0.0
            if ("beta", i, k) not in printed:
                assert be[i, k] == 0.0


@pytest.mark.parametrize("scheme", [oracle.RK3, oracle.SSPRK43, oracle.SSPRK54])
def test_rows_sum_to_one(scheme):
    # consistency of each stage (a convex combination): the printed 14-digit
    # SSPRK(5,4) row 5 sums to 1 - 1e-14; alpha_50 is renormalised so that the
    # exact sum of the binary64 coefficients is within one ulp of one.
    s, al, be = oracle.scheme_table(scheme)
    for i in range(1, s + 1):
        assert abs(math.fsum(al[i, :i]) - 1.0) <= 2.0**-52


@pytest.mark.parametrize("scheme,order,tol", [(oracle.RK3, 3, 1e-15), (oracle.SSPRK43, 3, 1e-15),
                                              (oracle.SSPRK54, 4, 2e-10)])
def test_order_conditions(scheme, order, tol):
    s, al, be = oracle.scheme_table(scheme)
    A, b = butcher(al, be)
    res = order_residuals(A, b)
    keys = ["b", "bc", "bc2", "bAc"] + (["bc3", "bcAc", "bAc2", "bAAc"] if order >= 4 else [])
    for k in keys:
        assert abs(res[k]) <= tol, (k, res[k])
    if order == 3:
        # a genuinely third-order scheme fails at least one fourth-order condition
        assert max(abs(res[k]) for k in ["bc3", "bcAc", "bAc2", "bAAc"]) > 1e-3


def test_stability_polynomials():
    s, al, be = oracle.scheme_table(oracle.SSPRK43)
    A, b = butcher(al, be)
    np.testing.assert_allclose(stability_poly(A, b), [1, 1, 1 / 2, 1 / 6, 1 / 48], atol=1e-15)
    s, al, be = oracle.scheme_table(oracle.SSPRK54)
    A, b = butcher(al, be)
    np.testing.assert_allclose(stability_poly(A, b)[:5], [1, 1, 1 / 2, 1 / 6, 1 / 24], atol=2e-10)
    assert abs(stability_poly(A, b)[5] - 0.0044777183) < 1e-9
    s, al, be = oracle.scheme_table(oracle.RK3)
    A, b = butcher(al, be)
    np.testing.assert_allclose(stability_poly(A, b), [1, 1, 1 / 2, 1 / 6], atol=1e-15)


def ssp_coefficient(al, be):
    r = np.inf
    s = al.shape[1]
    for i in range(1, s + 1):
        for k in range(i):
            if be[i, k] > 0:
                r = min(r, al[i, k] / be[i, k])
    return r


def test_ssp_coefficients_match_printed():
    g = {name: [v for kind, _, _, v in rows if kind == "ssp_cfl"][0]
         for name, rows in read_golden().items()}
    s, al, be = oracle.scheme_table(oracle.SSPRK43)
    assert abs(ssp_coefficient(al, be) - g["ssprk43"]) < 1e-15
    s, al, be = oracle.scheme_table(oracle.SSPRK54)
    assert abs(ssp_coefficient(al, be) - g["ssprk54"]) < 1e-9
    s, al, be = oracle.scheme_table(oracle.RK3)
    assert abs(ssp_coefficient(al, be) - 1.0) < 1e-15
