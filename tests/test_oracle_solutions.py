"""Pins of the oracle's whole scheme (Sect. 2) against exact solutions,
invariants and numbers printed in Sect. 4.5."""
import math

import numpy as np
import pytest

import oracle
from conftest import golden
from paper_1407_2052_amd import inputs


def paper_number(key):
    with open(golden("paper_numbers.txt")) as f:
        for line in f:
            if line.startswith(key + " "):
                return float(line.split()[1])
    raise KeyError(key)


def total(bs, v):
    return math.fsum(float(x) for b in range(bs.nb) for x in bs.interior(b)[v].ravel())


def fixed_dt(bs, T, cfl=0.4):
    _, cm = oracle.rhs(bs)
    dt0 = cfl / sum(cm[d] / bs.dx[0, d] for d in range(bs.ndim))
    n = int(math.ceil(T / dt0))
    return T / n, n


# --------------------------------------------------------------- invariants
@pytest.mark.parametrize("ndim,mhd", [(1, False), (2, False), (2, True), (3, True)])
def test_free_stream_is_preserved(ndim, mhd):
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(ndim, [8] * ndim, [4] * ndim)
    w = {"rho": 1.3, "p": 0.7, "vx": 0.4, "vy": -0.3, "vz": 0.2, "Bx": 0.9, "By": -0.5, "Bz": 0.25}
    bs = inputs.sample_blocks(ndim, mhd, 5 / 3, n, dx, xlo, nbr,
                              lambda X, Y, Z: {k: v + 0 * X for k, v in w.items()})
    L, _ = oracle.rhs(bs)
    for b in range(bs.nb):
        assert np.all(bs.interior(b, L[b]) == 0.0)
    out, _ = oracle.run(bs, oracle.SSPRK54, 3)
    ref = out.interior(0)[:, 0, 0, 0]
    for b in range(bs.nb):
        inner = out.interior(b)
        assert np.all(inner == ref[:, None, None, None])
    np.testing.assert_allclose(ref, bs.interior(0)[:, 0, 0, 0], rtol=1e-15)


@pytest.mark.parametrize("mhd", [False, True])
def test_periodic_conservation(mhd):
    bs = (inputs.orszag_tang_2d(32, 16) if mhd else inputs.hydro_random_2d(32, 16, seed=8))
    out, _ = oracle.run(bs, oracle.SSPRK54, 20)
    for v in range(bs.nvar):
        t0, t1 = total(bs, v), total(out, v)
        scale = math.fsum(abs(float(x)) for b in range(bs.nb) for x in bs.interior(b)[v].ravel())
        scale = max(scale, 1.0)
        assert abs(t1 - t0) <= 20 * 5 * 1e-15 * scale, (v, t0, t1)


def test_fixed_ghost_layers_are_constant_inputs():
    bs = inputs.sod(64)
    out, _ = oracle.run(bs, oracle.SSPRK54, 5)
    u0, u1 = bs.u[0], out.u[0]
    assert np.array_equal(u0[..., :3], u1[..., :3])
    assert np.array_equal(u0[..., -3:], u1[..., -3:])


@pytest.mark.parametrize("case", ["1d", "2d_mhd"])
def test_block_decomposition_is_bitwise_invisible(case):
    if case == "1d":
        one = inputs.density_wave_1d(64, nblocks=1)
        many = inputs.density_wave_1d(64, nblocks=8)
    else:
        one = inputs.orszag_tang_2d(32, 32)
        many = inputs.orszag_tang_2d(32, 8)
    a, dta = oracle.run(one, oracle.SSPRK54, 4)
    b, dtb = oracle.run(many, oracle.SSPRK54, 4)
    assert np.array_equal(dta, dtb)
    ua = a.interior(0)
    nbk = int(round(one.n[0, 0] / many.n[0, 0]))
    for blk in range(many.nb):
        ox = int(round((many.xlo[blk, 0] - one.xlo[0, 0]) / many.dx[blk, 0]))
        oy = int(round((many.xlo[blk, 1] - one.xlo[0, 1]) / many.dx[blk, 1])) if one.ndim > 1 else 0
        nx, ny = many.n[blk, 0], many.n[blk, 1]
        sub = ua[:, :, oy:oy + ny, ox:ox + nx]
        assert np.array_equal(sub, b.interior(blk)), blk
    assert nbk >= 1


# --------------------------------------------------------------- smooth flows
def density_wave_error(N, scheme, T=0.5):
    bs = inputs.density_wave_1d(N)
    dt, n = fixed_dt(bs, T)
    out, _ = oracle.run(bs, scheme, n, dt=dt)
    x = (np.arange(N) + 0.5) / N
    rho = out.interior(0)[0].ravel()
    m = out.interior(0)[1].ravel()
    E = out.interior(0)[2].ravel()
    v = m / rho
    p = (1.4 - 1.0) * (E - 0.5 * m * v)
    err = np.abs(rho - (1 + 0.2 * np.sin(2 * math.pi * (x - T)))).mean()
    return err, np.abs(v - 1).max(), np.abs(p - 1).max()


def test_density_wave_fifth_order_and_uniform_velocity_pressure():
    errs = []
    for N in (32, 64, 128):
        e, dv, dp = density_wave_error(N, oracle.SSPRK54)
        errs.append(e)
        assert dv < 1e-13 and dp < 1e-13
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(o > 4.8 for o in orders), orders


def test_density_wave_rk3_time_error_dominates():
    errs = [density_wave_error(N, oracle.RK3)[0] for N in (64, 128, 256)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] < 4.2 and orders[-1] > 2.8, orders


def alfven_errors(ndim, kvec, Ns, block_div=1):
    out_e = []
    for N in Ns:
        bs = inputs.circular_alfven(ndim, N, block=N // block_div, kvec=kvec)
        kn = math.sqrt(sum(k * k for k in kvec))
        T = 1.0 / kn
        dt, n = fixed_dt(bs, T)
        out, _ = oracle.run(bs, oracle.SSPRK54, n, dt=dt)
        e = np.mean([np.abs(out.interior(b) - bs.interior(b)).mean(axis=(1, 2, 3))
                     for b in range(bs.nb)], axis=0)
        out_e.append(e)
    return np.array(out_e)


def test_circular_alfven_wave_fifth_order_1d():
    E = alfven_errors(1, (1, 0, 0), (16, 32, 64))
    order = paper_number("alfven_observed_order_mp5_ssprk54")
    for v in (2, 3, 6, 7):
        o = np.log2(E[:-1, v] / E[1:, v])
        assert np.all(o > order - 0.2), (v, o)
    assert np.all(E[:, 0] < 1e-14)   # density stays uniform


def test_circular_alfven_wave_fifth_order_2d_oblique():
    E = alfven_errors(2, (1, 1, 0), (16, 32), block_div=2)
    for v in (2, 6, 7):
        o = math.log2(E[0, v] / E[1, v])
        assert o > 4.7, (v, o)


def test_linear_alfven_wave_phase():
    # small-amplitude wave: the Fourier phase of B_y after time T equals
    # -k v_A T exactly; the numerical phase error falls at high order.
    errs = []
    for N in (16, 32):
        bs = inputs.circular_alfven(1, N, amp=1e-6)
        T = 0.37
        dt, n = fixed_dt(bs, T)
        out, _ = oracle.run(bs, oracle.SSPRK54, n, dt=dt)
        def phase(b):
            by = b.interior(0)[6].ravel()
            return np.angle(np.fft.fft(by)[1])
        dphi = (phase(out) - phase(bs) + math.pi) % (2 * math.pi) - math.pi
        errs.append(abs(dphi - (-2 * math.pi * 1.0 * T)))
    assert errs[1] < 2e-6
    assert math.log2(errs[0] / errs[1]) > 4.5


# --------------------------------------------------------------- shocks
def exact_riemann(rl, ul, pl, rr, ur, pr, g, xi):
    """Exact solution of the Euler Riemann problem (Toro 1999, ch. 4) sampled
    at the similarity coordinates xi = (x - x0)/t."""
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fK(p, rk, pk, ck):
        if p > pk:
            A, B = 2 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f = fK(p, rl, pl, cl) + fK(p, rr, pr, cr) + ur - ul
        h = 1e-8 * p
        df = (fK(p + h, rl, pl, cl) + fK(p + h, rr, pr, cr) - fK(p - h, rl, pl, cl)
              - fK(p - h, rr, pr, cr)) / (2 * h)
        p_new = max(p - f / df, 1e-12)
        if abs(p_new - p) < 1e-14 * p:
            p = p_new
            break
        p = p_new
    us = 0.5 * (ul + ur) + 0.5 * (fK(p, rr, pr, cr) - fK(p, rl, pl, cl))
    out = np.zeros((3, len(xi)))
    for i, s in enumerate(xi):
        if s < us:   # left of contact
            if p > pl:
                rs = rl * ((p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1))
                S = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
                out[:, i] = (rl, ul, pl) if s < S else (rs, us, p)
            else:
                rs = rl * (p / pl) ** (1 / g)
                cs = cl * (p / pl) ** ((g - 1) / (2 * g))
                if s < ul - cl:
                    out[:, i] = (rl, ul, pl)
                elif s > us - cs:
                    out[:, i] = (rs, us, p)
                else:
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    out[:, i] = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if p > pr:
                rs = rr * ((p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1))
                S = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
                out[:, i] = (rr, ur, pr) if s > S else (rs, us, p)
            else:
                rs = rr * (p / pr) ** (1 / g)
                cs = cr * (p / pr) ** ((g - 1) / (2 * g))
                if s > ur + cr:
                    out[:, i] = (rr, ur, pr)
                elif s < us + cs:
                    out[:, i] = (rs, us, p)
                else:
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    out[:, i] = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out


def run_to_time(bs, T, cfl=0.4, scheme=oracle.SSPRK54):
    t, cur = 0.0, bs
    while t < T - 1e-14:
        _, cm = oracle.rhs(cur)
        dt = min(cfl / sum(cm[d] / cur.dx[0, d] for d in range(cur.ndim)), T - t)
        cur, _ = oracle.run(cur, scheme, 1, dt=dt)
        t += dt
    return cur


def test_exact_riemann_solver_textbook_values():
    # Sod star state (Toro 1999, Table 4.2, test 1): p* = 0.30313, u* = 0.92745
    sol = exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, np.array([0.9]))
    assert abs(sol[2, 0] - 0.30313) < 1e-5 and abs(sol[1, 0] - 0.92745) < 1e-5


def test_sod_against_exact_riemann_solution():
    errs = []
    for N in (100, 200, 400):
        bs = inputs.sod(N)
        out = run_to_time(bs, 0.2)
        u = out.interior(0)[:, 0, 0, :]
        rho, m, E = u
        v = m / rho
        p = 0.4 * (E - 0.5 * m * v)
        assert np.all(rho > 0) and np.all(p > 0)
        x = (np.arange(N) + 0.5) / N
        ex = exact_riemann(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (x - 0.5) / 0.2)
        errs.append(np.abs(rho - ex[0]).mean())
        # bounded oscillations: density stays within the data range (+/- 3%)
        assert rho.max() < 1.03 and rho.min() > 0.125 * 0.97
    assert errs[-1] < 6e-3
    o = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert all(0.5 < x < 1.6 for x in o), o


def test_brio_wu_contact_overshoot_matches_paper():
    N = int(paper_number("brio_wu_cells"))
    bs = inputs.brio_wu(N)
    out = run_to_time(bs, paper_number("brio_wu_t_end"), cfl=paper_number("brio_wu_courant"))
    x = out.xlo[0, 0] + (np.arange(N) + 0.5) * out.dx[0, 0]
    rho = out.interior(0)[0].ravel()
    # contact: steepest density drop between the compound wave and the
    # slow shock; plateau: median density just left of it
    region = (x > 0.0) & (x < 0.25)
    idx = np.where(region)[0]
    drop = np.argmin(np.diff(rho[idx]))
    xc = x[idx[drop]]
    plateau = np.median(rho[(x > xc - 0.12) & (x < xc - 0.03)])
    peak = rho[(x > xc - 0.03) & (x <= xc)].max()
    over = 100 * (peak / plateau - 1)
    ref = paper_number("brio_wu_mp5_fd_density_overshoot_percent")
    assert abs(over - ref) < 1.0, over
