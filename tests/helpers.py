"""Shared test helpers: seeded smooth states on arbitrary block lists, GPU
runners through the C ABI, and comparison norms."""
import math

import numpy as np

from paper_1407_2052_amd import inputs


def smooth_fields(ndim, mhd, seed, amp=0.05, nmodes=2, base=None):
    """Closure sampling seeded random-phase periodic fields (unit box)."""
    rng = np.random.default_rng(seed)
    names = ["rho", "vx", "vy", "vz", "p"] + (["Bx", "By", "Bz"] if mhd else [])
    b0 = {"rho": 1.0, "vx": 0.3, "vy": -0.2, "vz": 0.1, "p": 1.0, "Bx": 0.8, "By": 0.4, "Bz": -0.3}
    if base:
        b0.update(base)
    modes = {k: [(rng.integers(1, 3, size=3), rng.uniform(0, 2 * math.pi)) for _ in range(nmodes)]
             for k in names}

    def f(X, Y, Z):
        out = {}
        for k in names:
            acc = b0[k]
            for kv, ph in modes[k]:
                acc = acc + amp * np.sin(2 * math.pi * (kv[0] * X + kv[1] * Y + kv[2] * Z) + ph)
            out[k] = acc
        return out
    return f


def strip_blocks(ndim, mhd, xs, ny=1, nz=1, seed=0, periodic=True, gamma=5 / 3, amp=0.05):
    """Blocks of widths xs (along x) side by side, each ny x nz, on a box of
    size sum(xs) x ny x nz cells with dx = 1/sum(xs) (ragged block sizes)."""
    nb = len(xs)
    N = sum(xs)
    dxv = 1.0 / N
    n = np.ones((nb, 3), np.int32)
    dx = np.ones((nb, 3))
    xlo = np.zeros((nb, 3))
    nbr = -np.ones((nb, 6), np.int32)
    x0 = 0
    for b, w in enumerate(xs):
        n[b] = [w, ny if ndim > 1 else 1, nz if ndim > 2 else 1]
        dx[b] = [dxv, dxv if ndim > 1 else 1.0, dxv if ndim > 2 else 1.0]
        xlo[b] = [x0 * dxv, 0.0, 0.0]
        x0 += w
        if periodic or b > 0:
            nbr[b, 0] = (b - 1) % nb
        if periodic or b < nb - 1:
            nbr[b, 1] = (b + 1) % nb
        for d in range(1, ndim):
            if periodic:
                nbr[b, 2 * d] = b
                nbr[b, 2 * d + 1] = b
    return inputs.sample_blocks(ndim, mhd, gamma, n, dx, xlo, nbr, smooth_fields(ndim, mhd, seed, amp))


def rel_l1(a_blocks, b_blocks, bs, v):
    """sum |a - b| / sum |b| over the interiors, variable v (b = reference)."""
    num = sum(float(np.abs(bs.interior(i, a)[v] - bs.interior(i, b)[v]).sum()) for i, (a, b) in
              enumerate(zip(a_blocks, b_blocks)))
    den = sum(float(np.abs(bs.interior(i, b)[v]).sum()) for i, b in enumerate(b_blocks))
    return num, den
