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


# ---------------------------------------------------------------------------
# Summaries of a full-size state, so that a stored oracle run can be compared
# with a GPU run without storing the whole state.
# ---------------------------------------------------------------------------
def state_summary(bs, u_blocks, seed=12345, nsample=4096):
    """Per block and variable: L1 = sum |U|, S = sum U and P = sum w U with
    seeded weights w ~ U(-1, 1) per interior cell (|P_a - P_b| <= ||U_a -
    U_b||_1, so P catches localised differences); plus the state at nsample
    seeded interior cells (block, z, y, x)."""
    nb, nv = bs.nb, bs.nvar
    l1 = np.zeros((nb, nv))
    s = np.zeros((nb, nv))
    p = np.zeros((nb, nv))
    for b in range(nb):
        x = bs.interior(b, u_blocks[b])
        w = np.random.default_rng([seed, b]).uniform(-1.0, 1.0, size=x.shape[1:])
        l1[b] = np.abs(x).reshape(nv, -1).sum(axis=1)
        s[b] = x.reshape(nv, -1).sum(axis=1)
        p[b] = (x * w[None]).reshape(nv, -1).sum(axis=1)
    rng = np.random.default_rng(seed)
    idx = np.zeros((nsample, 4), np.int64)
    val = np.zeros((nsample, nv))
    for q in range(nsample):
        b = int(rng.integers(0, nb))
        z, y, xx = (int(rng.integers(0, bs.n[b, d])) if d < bs.ndim else 0 for d in (2, 1, 0))
        idx[q] = (b, z, y, xx)
        val[q] = bs.interior(b, u_blocks[b])[:, z, y, xx]
    return {"l1": l1, "sum": s, "proj": p, "sample_idx": idx, "sample_val": val}


def input_digest(bs):
    """sha256 of every block's padded state (identifies the generated input)."""
    import hashlib
    h = hashlib.sha256()
    for x in bs.u:
        h.update(np.ascontiguousarray(x).tobytes())
    return h.hexdigest()
