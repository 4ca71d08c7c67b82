"""Pins of the oracle's reverse mode (local dual-number Jacobians of each
cell's flux and each reconstruction, applied transposed and scattered, the
c_max derivative delivered to the maximising cell, ghost adjoints returned
to the owner cells of periodic faces and kept as boundary-data adjoints on
fixed faces).

Independent checks: the dot-product identity <lam_0, dU_0> = <lam_N, J dU_0>
against the forward-mode JVP (which propagates tangents through the whole
integration and shares none of the reverse mode's transposition or
scattering), tangents placed in the fixed ghost layers included; central
differences of the forward map on states whose branch fingerprints agree at
+-h; and the full Jacobian of a tiny grid, entry by entry."""
import math

import numpy as np
import pytest

import oracle
from paper_1407_2052_amd import inputs
from test_oracle_jvp import random_mhd, smooth_hydro_2d


def dot(a, b):
    return math.fsum(float(np.vdot(x, y)) for x, y in zip(a, b))


def fixed_dt(bs, cfl=0.3):
    _, cm = oracle.rhs(bs)
    return cfl / max(sum(cm[d] / bs.dx[b, d] for d in range(bs.ndim)) for b in range(bs.nb))


def random_interior(bs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(bs.nb):
        x = np.zeros(bs.padded_shape(b))
        bs.interior(b, x)[...] = rng.normal(size=bs.interior(b).shape)
        out.append(x)
    return out


def face_ghost_mask(bs, b):
    """True on the face ghosts of fixed faces (edges and corners excluded)."""
    m = np.zeros(bs.u[b].shape[1:], dtype=bool)
    P = m.shape[::-1]   # (Px, Py, Pz)
    for d in range(bs.ndim):
        for side in (0, 1):
            if bs.nbr[b, 2 * d + side] >= 0:
                continue
            sl = []
            for e in (2, 1, 0):
                if e >= bs.ndim:
                    sl.append(slice(0, 1))
                elif e == d:
                    sl.append(slice(0, 3) if side == 0 else slice(P[e] - 3, P[e]))
                else:
                    sl.append(slice(3, P[e] - 3))
            m[tuple(sl)] = True
    return m


def random_with_ghosts(bs, seed):
    """Random interior and fixed-face ghost entries (smoothness is not needed
    for a dot-product test of a piecewise-linear-in-the-tangent map)."""
    rng = np.random.default_rng(seed)
    out = random_interior(bs, seed)
    for b in range(bs.nb):
        g = face_ghost_mask(bs, b)
        out[b][:, g] = rng.normal(size=(bs.nvar, int(g.sum())))
    return out


def sod_like(N=32, blocks=2):
    """Smooth 1D Euler data with fixed faces on both ends (no shock: every
    branch of the limiter is away from its kinks)."""
    n, dx, xlo, nbr, _ = inputs.uniform_blocks(1, [N], [N // blocks], periodic=False)
    tp = 2 * math.pi
    return inputs.sample_blocks(1, False, 1.4, n, dx, xlo, nbr, lambda X, Y, Z: {
        "rho": 1 + 0.2 * np.sin(tp * X + 0.4) + 0.05 * np.cos(3 * tp * X), "vx": 0.4 + 0.1 * np.cos(tp * X),
        "p": 1 + 0.1 * np.sin(tp * X + 1.0)})


def mhd2d_mixed_faces():
    """2D MHD, 2 x 2 blocks: periodic along x, fixed faces along y."""
    bs = random_mhd(2, 16, 8, seed=11)
    for b in range(bs.nb):
        for side in (0, 1):
            j = bs.nbr[b, 2 + side]
            yb = int(round(bs.xlo[b, 1] * 16)) // 8
            if (side == 0 and yb == 0) or (side == 1 and yb == 1):
                bs.nbr[b, 2 + side] = -1
    return bs


CASES = {
    "hydro2d_ssprk54": (smooth_hydro_2d, oracle.SSPRK54, 3, oracle.MP5),
    "hydro2d_rk3": (smooth_hydro_2d, oracle.RK3, 3, oracle.MP5),
    "mhd2d_ssprk43": (lambda: random_mhd(2, 16, 8, 5), oracle.SSPRK43, 2, oracle.MP5),
    "mhd1d_ssprk54": (lambda: random_mhd(1, 32, 16, 6), oracle.SSPRK54, 4, oracle.MP5),
    "mhd3d_ssprk54": (lambda: random_mhd(3, 8, 8, 7), oracle.SSPRK54, 1, oracle.MP5),
    "lim03_mhd2d_rk3": (lambda: random_mhd(2, 16, 8, 8), oracle.RK3, 3, oracle.LIM03),
    "fixed_hydro1d": (sod_like, oracle.SSPRK54, 4, oracle.MP5),
    "fixed_mixed_mhd2d": (mhd2d_mixed_faces, oracle.SSPRK54, 2, oracle.MP5),
    "fixed_lim03_hydro1d": (sod_like, oracle.RK3, 4, oracle.LIM03),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_dot_product_against_the_jvp(case):
    gen, scheme, nsteps, rec = CASES[case]
    bs = gen()
    with oracle.use_recon(rec):
        dt = fixed_dt(bs)
        tang = random_with_ghosts(bs, 3)
        lam_n = random_interior(bs, 4)
        _, du = oracle.run_jvp(bs, tang, scheme, nsteps, dt)
        lam0 = oracle.run_vjp(bs, lam_n, scheme, nsteps, dt)
    lhs = dot(lam0, tang)
    rhs = math.fsum(float(np.vdot(bs.interior(b, lam_n[b]), bs.interior(b, du[b]))) for b in range(bs.nb))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs), (lhs, rhs, (lhs - rhs) / rhs)
    # ghosts: boundary-data adjoint on fixed faces only, zero elsewhere
    for b in range(bs.nb):
        g = np.ones(bs.u[b].shape[1:], dtype=bool)
        bs.interior(b, g[None])[...] = False
        g &= ~face_ghost_mask(bs, b)
        assert np.all(lam0[b][:, g] == 0.0)
    if case.startswith("fixed"):
        assert any(np.any(lam0[b][:, face_ghost_mask(bs, b)] != 0.0) for b in range(bs.nb))


def test_full_jacobian_of_a_tiny_grid_entry_by_entry():
    """8-cell periodic 1D MHD, 2 SSPRK(5,4) steps: every entry of lam_0 equals
    <lam_N, J e_k> from one JVP per input k."""
    bs = random_mhd(1, 8, 8, seed=9)
    dt = fixed_dt(bs)
    lam_n = random_interior(bs, 10)
    lam0 = oracle.run_vjp(bs, lam_n, oracle.SSPRK54, 2, dt)[0]
    ref = np.zeros_like(lam0)
    for v in range(bs.nvar):
        for i in range(8):
            e = np.zeros(bs.padded_shape(0))
            e[v, 0, 0, i + 3] = 1.0
            _, du = oracle.run_jvp(bs, [e], oracle.SSPRK54, 2, dt)
            ref[v, 0, 0, i + 3] = float(np.vdot(bs.interior(0, lam_n[0]), bs.interior(0, du[0])))
    scale = np.abs(ref).max()
    assert np.abs(lam0 - ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("which", ["interior", "fixed_ghost"])
def test_gradient_matches_central_differences(which):
    """J = <w, U_N> on the fixed-face 1D case: a gradient entry against a
    central difference of the forward map (branch fingerprints equal at
    +-h, so the difference quotient crosses no kink)."""
    bs = sod_like()
    dt = fixed_dt(bs)
    nsteps = 3
    w = random_interior(bs, 21)
    lam0 = oracle.run_vjp(bs, w, oracle.SSPRK54, nsteps, dt)
    if which == "interior":
        b, idx = 1, (2, 0, 0, 3 + 5)
    else:
        b, idx = 0, (0, 0, 0, 1)    # density in the second ghost cell of the left fixed face
    h = 1e-6

    def J(sign):
        x = bs.copy()
        x.u[b][idx] += sign * h
        out, _ = oracle.run(x, oracle.SSPRK54, nsteps, dt=dt)
        return math.fsum(float(np.vdot(out.interior(q), x.interior(q, w[q]))) for q in range(bs.nb)), x

    Jp, xp = J(+1)
    Jm, xm = J(-1)
    assert oracle.run_branch_hash(xp, oracle.SSPRK54, nsteps, dt) == oracle.run_branch_hash(xm, oracle.SSPRK54, nsteps, dt)
    fd = (Jp - Jm) / (2 * h)
    assert abs(fd - lam0[b][idx]) <= 1e-6 * max(abs(fd), 1e-3), (fd, lam0[b][idx])
