"""Seeded synthetic inputs: block lists with ghost-padded conserved states.

This module only *builds inputs*: block geometry, neighbour tables and the
initial conserved state sampled point-wise at cell centres (the
finite-difference point-value interpretation of Sect. 2.1).  It holds none of
the scheme's arithmetic (no primitive recovery, flux, speed, reconstruction
or time stepping) and is the only module that both the HIP path's tests and
the oracle consume.

Layout of one block (the public C-ABI layout): a float64 array of shape
``(nvar, P_z, P_y, P_x)``, C-contiguous (x fastest), with ``P_d = n_d + 6``
for active directions and 1 otherwise (3 ghost layers on each side).
Variable order: hydro ``(rho, m_1..m_ndim, E)``; MHD
``(rho, m_x, m_y, m_z, E, B_x, B_y, B_z)``.

Workloads (Sect. 4.5 and the benchmark set):
  * 1D density wave, 512 cells, periodic (Euler, gamma 1.4);
  * 2D Orszag-Tang-type smooth MHD data, 512^2 as 1024 blocks of 16^2;
  * 3D MHD uneven blocks 8^3/16^3/32^3 (4:2:1), fixed ghosts from an 8-mode
    field;
  * 2D hydro random density (8 modes), 256^2 as 256 blocks of 16^2;
  * 3D MHD turbulence-like 16-mode perturbations, 256^3 as 4096 blocks of
    16^3;
  * analytic test states: circularly polarised and linear Alfven waves
    (Sect. 4.5.1), Sod and Brio-Wu shock tubes (Sect. 4.5.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

NG = 3


def nvar_of(ndim: int, mhd) -> int:
    """mhd: False/0 hydro, True/1 ideal MHD, 2 GLM-MHD (MHD + psi)."""
    return 9 if mhd == 2 else 8 if mhd else 2 + ndim


@dataclasses.dataclass
class BlockSet:
    ndim: int
    mhd: bool
    gamma: float
    n: np.ndarray        # (nb, 3) int32, 1 for inactive directions
    dx: np.ndarray       # (nb, 3) float64
    xlo: np.ndarray      # (nb, 3) float64, lower face of the first interior cell
    nbr: np.ndarray      # (nb, 6) int32, -1 = fixed (caller-filled) ghosts
    u: List[np.ndarray]  # per block (nvar, Pz, Py, Px) float64

    @property
    def nb(self) -> int:
        return len(self.u)

    @property
    def nvar(self) -> int:
        return nvar_of(self.ndim, self.mhd)

    def interior_cells(self) -> int:
        return int(np.prod(self.n, axis=1).sum())

    def interior(self, b: int, arr: Optional[np.ndarray] = None) -> np.ndarray:
        """View of the interior of block b (of `arr`, default the state)."""
        a = self.u[b] if arr is None else arr
        sl = [slice(None)]
        for d in (2, 1, 0):
            sl.append(slice(NG, NG + self.n[b, d]) if d < self.ndim else slice(0, 1))
        return a[tuple(sl)]

    def copy(self) -> "BlockSet":
        return dataclasses.replace(self, u=[x.copy() for x in self.u], n=self.n.copy(),
                                   dx=self.dx.copy(), xlo=self.xlo.copy(), nbr=self.nbr.copy())

    def padded_shape(self, b: int) -> Tuple[int, int, int, int]:
        P = [int(self.n[b, d]) + 2 * NG if d < self.ndim else 1 for d in range(3)]
        return (self.nvar, P[2], P[1], P[0])


# ---------------------------------------------------------------------------
# Conserved state from primitive fields (definition of the initial data:
# m = rho v, E = p/(gamma-1) + rho v^2/2 [+ B^2/2], Sect. 3.2 and eq. frace).
# ---------------------------------------------------------------------------
PrimFields = Dict[str, np.ndarray]   # keys rho, vx, vy, vz, p, Bx, By, Bz[, psi]


def conserved_from_prims(ndim: int, mhd: bool, gamma: float, w: PrimFields) -> np.ndarray:
    rho = w["rho"]
    v = [w.get("vx", 0.0 * rho), w.get("vy", 0.0 * rho), w.get("vz", 0.0 * rho)]
    p = w["p"]
    nc = 3 if mhd else ndim
    out = [rho]
    kin = 0.0 * rho
    for k in range(nc):
        out.append(rho * v[k])
        kin = kin + rho * v[k] * v[k]
    E = p / (gamma - 1.0) + 0.5 * kin
    if mhd:
        B = [w.get("Bx", 0.0 * rho), w.get("By", 0.0 * rho), w.get("Bz", 0.0 * rho)]
        E = E + 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2])
        out.append(E)
        out.extend(B)
        if mhd == 2:   # GLM: the divergence-cleaning potential psi
            out.append(w.get("psi", 0.0 * rho))
    else:
        out.append(E)
    return np.ascontiguousarray(np.stack([np.broadcast_to(x, rho.shape) for x in out]))


# ---------------------------------------------------------------------------
# Geometry helpers
# ---------------------------------------------------------------------------
def uniform_blocks(ndim: int, cells: Sequence[int], block: Sequence[int],
                   lo: Sequence[float] = (0.0, 0.0, 0.0), hi: Sequence[float] = (1.0, 1.0, 1.0),
                   periodic: bool = True):
    """Tile a box of `cells` into blocks of `block` cells, lexicographic block
    order with x fastest.  Returns (n, dx, xlo, nbr, block_index_grid)."""
    cells = list(cells) + [1] * (3 - len(cells))
    block = list(block) + [1] * (3 - len(block))
    nbd = [cells[d] // block[d] if d < ndim else 1 for d in range(3)]
    for d in range(ndim):
        if cells[d] % block[d]:
            raise ValueError("cells must be a multiple of the block size")
    dxs = [(hi[d] - lo[d]) / cells[d] if d < ndim else 1.0 for d in range(3)]
    nb = nbd[0] * nbd[1] * nbd[2]
    n = np.ones((nb, 3), np.int32)
    dx = np.ones((nb, 3), np.float64)
    xlo = np.zeros((nb, 3), np.float64)
    nbr = -np.ones((nb, 6), np.int32)
    grid = np.arange(nb).reshape(nbd[2], nbd[1], nbd[0])
    for bz in range(nbd[2]):
        for by in range(nbd[1]):
            for bx in range(nbd[0]):
                b = grid[bz, by, bx]
                c = (bx, by, bz)
                for d in range(3):
                    n[b, d] = block[d] if d < ndim else 1
                    dx[b, d] = dxs[d]
                    xlo[b, d] = lo[d] + c[d] * block[d] * dxs[d] if d < ndim else 0.0
                for d in range(ndim):
                    for side, step in ((0, -1), (1, 1)):
                        cc = list(c)
                        cc[d] += step
                        if 0 <= cc[d] < nbd[d]:
                            nbr[b, 2 * d + side] = grid[cc[2], cc[1], cc[0]]
                        elif periodic:
                            cc[d] %= nbd[d]
                            nbr[b, 2 * d + side] = grid[cc[2], cc[1], cc[0]]
    return n, dx, xlo, nbr, grid


def cell_centres(ndim: int, n: np.ndarray, dx: np.ndarray, xlo: np.ndarray):
    """Cell-centre coordinates of the padded block, broadcastable (z, y, x)."""
    axes = []
    for d in range(3):
        if d < ndim:
            i = np.arange(-NG, n[d] + NG, dtype=np.float64)
            axes.append(xlo[d] + (i + 0.5) * dx[d])
        else:
            axes.append(np.zeros(1))
    X = axes[0][None, None, :]
    Y = axes[1][None, :, None]
    Z = axes[2][:, None, None]
    return X, Y, Z


def sample_blocks(ndim: int, mhd: bool, gamma: float, n, dx, xlo, nbr,
                  prim_fn: Callable[[np.ndarray, np.ndarray, np.ndarray], PrimFields]) -> BlockSet:
    """Sample primitive fields point-wise at every padded cell centre."""
    us = []
    for b in range(len(n)):
        X, Y, Z = cell_centres(ndim, n[b], dx[b], xlo[b])
        w = prim_fn(X, Y, Z)
        shape = np.broadcast_shapes(X.shape, Y.shape, Z.shape)
        w = {k: np.broadcast_to(np.asarray(v, np.float64), shape) for k, v in w.items()}
        us.append(conserved_from_prims(ndim, mhd, gamma, w))
    return BlockSet(ndim, mhd, gamma, n.astype(np.int32), dx, xlo, nbr.astype(np.int32), us)


# ---------------------------------------------------------------------------
# Seeded Fourier-mode perturbations on the periodic unit box
# ---------------------------------------------------------------------------
def random_modes(rng: np.random.Generator, ndim: int, nmodes: int, kmax: int = 4):
    ks, amps, phases = [], [], []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=ndim)
        if not np.any(k):
            continue
        ks.append(np.concatenate([k, np.zeros(3 - ndim, np.int64)]))
        amps.append(rng.uniform(0.5, 1.0))
        phases.append(rng.uniform(0.0, 2.0 * math.pi))
    return np.array(ks), np.array(amps), np.array(phases)


def lattice_modes(N: Sequence[int], ks, weights, phases) -> np.ndarray:
    """sum_m weights[m] * sin(2 pi k_m . x + phi_m) at the cell centres of the
    periodic lattice N (x = (i + 1/2)/N per axis), via separable complex
    exponentials: the (y, z) factors of all modes sharing k_x are summed
    first, then one real outer product per distinct k_x.
    Returns an array (Nz, Ny, Nx)."""
    N = list(N) + [1] * (3 - len(N))
    e = []
    for d in range(3):
        x = (np.arange(N[d]) + 0.5) / N[d]
        e.append({int(k): np.exp(2j * math.pi * k * x) for k in np.unique(ks[:, d])})
    out = np.zeros((N[2], N[1], N[0]))
    for kx in np.unique(ks[:, 0]):
        yz = np.zeros((N[2], N[1]), np.complex128)
        for k, wgt, ph in zip(ks, weights, phases):
            if int(k[0]) == int(kx):
                yz += wgt * np.exp(1j * ph) * (e[2][int(k[2])][:, None] * e[1][int(k[1])][None, :])
        ex = e[0][int(kx)]
        # Im(yz * ex) = Re(yz) Im(ex) + Im(yz) Re(ex)
        out += yz.real[:, :, None] * ex.imag[None, None, :]
        out += yz.imag[:, :, None] * ex.real[None, None, :]
    return out


def perturbation(rng, N, ndim, nmodes, amplitude):
    """amplitude * sum_m a_m sin(2 pi k_m.x + phi_m) / sum_m a_m (|.| <= amplitude)."""
    ks, a, ph = random_modes(rng, ndim, nmodes)
    return amplitude * lattice_modes(N, ks, a / a.sum(), ph)


def solenoidal_perturbation(rng, N, ndim, nmodes, amplitude):
    """Vector field amplitude * sum_m a_m e_m sin(2 pi k_m.x + phi_m) / sum a_m
    with unit e_m perpendicular to k_m (divergence-free)."""
    ks, a, ph = random_modes(rng, ndim, nmodes)
    comps = [np.zeros(([1] * (3 - len(N))) + list(N)[::-1]) for _ in range(3)]
    for k, am, p in zip(ks, a, ph):
        r = rng.normal(size=3)
        kf = k.astype(np.float64)
        r -= kf * (r @ kf) / (kf @ kf)
        r /= np.linalg.norm(r)
        field = lattice_modes(N, k[None, :], np.array([am / a.sum()]), np.array([p]))
        for c in range(3):
            comps[c] = comps[c] + amplitude * r[c] * field
    return comps


def blocks_from_lattice(ndim: int, mhd: bool, gamma: float, fields: PrimFields,
                        N: Sequence[int], origins: np.ndarray, sizes: np.ndarray,
                        nbr: np.ndarray) -> BlockSet:
    """Cut padded blocks (with wrap-around) out of periodic lattice fields."""
    N3 = list(N) + [1] * (3 - len(N))
    nb = len(origins)
    n = np.ones((nb, 3), np.int32)
    dx = np.ones((nb, 3))
    xlo = np.zeros((nb, 3))
    us = []
    for b in range(nb):
        idx = []
        for d in range(3):
            if d < ndim:
                n[b, d] = sizes[b, d]
                dx[b, d] = 1.0 / N3[d]
                xlo[b, d] = origins[b, d] / N3[d]
                idx.append((origins[b, d] + np.arange(-NG, sizes[b, d] + NG)) % N3[d])
            else:
                idx.append(np.zeros(1, np.int64))
        sel = np.ix_(idx[2], idx[1], idx[0])
        w = {k: v[sel] for k, v in fields.items()}
        us.append(conserved_from_prims(ndim, mhd, gamma, w))
    return BlockSet(ndim, mhd, gamma, n, dx, xlo, nbr.astype(np.int32), us)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def density_wave_1d(N: int = 512, nblocks: int = 1, gamma: float = 1.4,
                    amp: float = 0.2, v: float = 1.0, p: float = 1.0) -> BlockSet:
    """rho = 1 + amp sin(2 pi x), v, p uniform, periodic [0,1)."""
    n, dx, xlo, nbr, _ = uniform_blocks(1, [N], [N // nblocks])
    return sample_blocks(1, False, gamma, n, dx, xlo, nbr, lambda X, Y, Z: {
        "rho": 1.0 + amp * np.sin(2 * math.pi * X), "vx": v + 0 * X, "p": p + 0 * X})


def orszag_tang_2d(N: int = 512, block: int = 16, gamma: float = 5.0 / 3.0) -> BlockSet:
    """Smooth Orszag-Tang-type data on the periodic unit square."""
    n, dx, xlo, nbr, _ = uniform_blocks(2, [N, N], [block, block])
    s4p = math.sqrt(4 * math.pi)

    def f(X, Y, Z):
        one = np.ones(np.broadcast_shapes(X.shape, Y.shape))
        return {"rho": 25.0 / (36.0 * math.pi) * one, "p": 5.0 / (12.0 * math.pi) * one,
                "vx": -np.sin(2 * math.pi * Y) * one, "vy": np.sin(2 * math.pi * X) * one,
                "Bx": -np.sin(2 * math.pi * Y) / s4p * one,
                "By": np.sin(4 * math.pi * X) / s4p * one}
    return sample_blocks(2, True, gamma, n, dx, xlo, nbr, f)


def uneven_sizes(nblocks: int) -> List[int]:
    """Sizes 32^3 : 16^3 : 8^3 in ratio 1 : 2 : 4 by count, largest first."""
    n32 = nblocks // 7
    n16 = 2 * n32
    n8 = nblocks - n32 - n16
    return [32] * n32 + [16] * n16 + [8] * n8


def uneven_3d(nblocks: int = 4096, seed: int = 3, N: int = 256, gamma: float = 5.0 / 3.0,
              amplitude: float = 0.1, nmodes: int = 8) -> BlockSet:
    """3D ideal MHD, `nblocks` independent blocks of 32^3/16^3/8^3 (1:2:4),
    origins on the 1/N lattice of the periodic unit cube, every face fixed
    (ghosts sampled from the same field).  Background rho = 1, p = 1,
    B = (1, 0, 0), v = 0; each primitive field carries its own `nmodes`-mode
    perturbation of amplitude `amplitude`."""
    rng = np.random.default_rng(seed)
    sizes1 = uneven_sizes(nblocks)
    names = ["rho", "vx", "vy", "vz", "p", "Bx", "By", "Bz"]
    base = {"rho": 1.0, "vx": 0.0, "vy": 0.0, "vz": 0.0, "p": 1.0, "Bx": 1.0, "By": 0.0, "Bz": 0.0}
    fields = {k: base[k] + perturbation(rng, [N, N, N], 3, nmodes, amplitude) for k in names}
    origins = np.stack([rng.integers(0, N, size=nblocks) for _ in range(3)], axis=1)
    sizes = np.array([[s, s, s] for s in sizes1], np.int64)
    nbr = -np.ones((nblocks, 6), np.int32)
    return blocks_from_lattice(3, True, gamma, fields, [N, N, N], origins, sizes, nbr)


def hydro_random_2d(N: int = 256, block: int = 16, seed: int = 4, gamma: float = 1.4,
                    amplitude: float = 0.05, nmodes: int = 8) -> BlockSet:
    """2D Euler, rho = 1 + 8-mode perturbation, v = 0, p = 1, periodic."""
    rng = np.random.default_rng(seed)
    drho = perturbation(rng, [N, N], 2, nmodes, amplitude)
    n, dx, xlo, nbr, grid = uniform_blocks(2, [N, N], [block, block])
    origins = np.stack([np.rint(xlo[:, 0] * N).astype(np.int64),
                        np.rint(xlo[:, 1] * N).astype(np.int64), np.zeros(len(n), np.int64)], 1)
    fields = {"rho": 1.0 + drho, "p": np.ones_like(drho)}
    return blocks_from_lattice(2, False, gamma, fields, [N, N], origins, n.astype(np.int64), nbr)


def hydro_target_density(N: int = 256, block: int = 16, seed: int = 40,
                         amplitude: float = 0.05, nmodes: int = 8) -> List[np.ndarray]:
    """Target density (interior arrays per block) drawn with the same recipe."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + perturbation(rng, [N, N], 2, nmodes, amplitude)
    n, dx, xlo, nbr, grid = uniform_blocks(2, [N, N], [block, block])
    out = []
    for b in range(len(n)):
        ox, oy = int(round(xlo[b, 0] * N)), int(round(xlo[b, 1] * N))
        out.append(np.ascontiguousarray(rho[:, oy:oy + block, ox:ox + block]))
    return out


def mhd_turbulence_3d(N: int = 256, block: int = 16, seed: int = 5, gamma: float = 5.0 / 3.0,
                      amplitude: float = 0.1, nmodes: int = 16) -> BlockSet:
    """3D ideal MHD, periodic N^3 in blocks of block^3; rho = 1, p = 0.5,
    B = (1, 0, 0) (plasma beta 2p/B^2 = 1), solenoidal `nmodes`-mode velocity
    and magnetic perturbations of amplitude `amplitude`."""
    rng = np.random.default_rng(seed)
    dv = solenoidal_perturbation(rng, [N, N, N], 3, nmodes, amplitude)
    dB = solenoidal_perturbation(rng, [N, N, N], 3, nmodes, amplitude)
    one = np.ones((N, N, N))
    fields = {"rho": one, "p": 0.5 * one, "vx": dv[0], "vy": dv[1], "vz": dv[2],
              "Bx": 1.0 + dB[0], "By": dB[1], "Bz": dB[2]}
    n, dx, xlo, nbr, grid = uniform_blocks(3, [N, N, N], [block, block, block])
    origins = np.rint(xlo * N).astype(np.int64)
    return blocks_from_lattice(3, True, gamma, fields, [N, N, N], origins, n.astype(np.int64), nbr)


def circular_alfven(ndim: int, N: int, block: Optional[int] = None, amp: float = 0.1,
                    rho0: float = 1.0, p0: float = 0.1, gamma: float = 5.0 / 3.0,
                    kvec: Tuple[int, int, int] = (1, 0, 0), t: float = 0.0,
                    direction: int = +1, glm: bool = False) -> BlockSet:
    """Circularly polarised Alfven wave (Sect. 4.5.1, eq. alfven) on the
    periodic unit box, wave vector 2 pi kvec, v_A = 1 along k, amplitude
    `amp`, propagating along +k (direction=+1) or -k."""
    k = np.array(kvec, np.float64)[:ndim]
    kn = np.linalg.norm(k)
    khat = np.zeros(3); khat[:ndim] = k / kn
    # orthonormal frame (khat, e1, e2)
    trial = np.array([0.0, 0.0, 1.0]) if abs(khat[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(trial, khat); e1 /= np.linalg.norm(e1)
    e2 = np.cross(khat, e1)
    cells = [N] * ndim
    n, dx, xlo, nbr, _ = uniform_blocks(ndim, cells, [block or N] * ndim)
    sq = math.sqrt(rho0)
    vA = 1.0

    def f(X, Y, Z):
        shape = np.broadcast_shapes(X.shape, Y.shape, Z.shape)
        xs = [X, Y, Z]
        phase = 0.0 * np.zeros(shape)
        for d in range(ndim):
            phase = phase + 2 * math.pi * kvec[d] * xs[d]
        phase = phase - direction * 2 * math.pi * kn * vA * t
        vpar = [amp * np.sin(phase), amp * np.cos(phase)]
        v = [vpar[0] * e1[c] + vpar[1] * e2[c] for c in range(3)]
        B = [sq * vA * khat[c] - direction * sq * (vpar[0] * e1[c] + vpar[1] * e2[c])
             for c in range(3)]
        one = np.ones(shape)
        return {"rho": rho0 * one, "p": p0 * one, "vx": v[0] * one, "vy": v[1] * one,
                "vz": v[2] * one, "Bx": B[0] * one, "By": B[1] * one, "Bz": B[2] * one}
    return sample_blocks(ndim, 2 if glm else True, gamma, n, dx, xlo, nbr, f)


def alfven_whistler(ndim: int, N: int, d: float, branch: int = -1, kvec: Tuple[int, int, int] = (1, 0, 0),
                    block: Optional[int] = None, amp: float = 0.1, B0: float = 1.0, p0: float = 0.1,
                    gamma: float = 5.0 / 3.0):
    """Circularly polarised Alfven-whistler wave of Hall MHD (Sect. 4.5.3)
    with rho = 1, ion inertial length d (= eta_h at rho = 1), along the wave
    vector 2 pi kvec on the periodic unit box.  In the frame (k, e1, e2) the
    transverse field b = b1 + i b2 = amp exp(i(k.x - w t)) and velocity
    u = -(|k| B0 / w) b solve Hall MHD exactly; w = |k| v with v = B0 (-d|k|/2
    + branch sqrt(1 + (d|k|/2)^2)): branch +1 the ion-cyclotron branch
    (w > 0), -1 the whistler branch (w < 0, phase speed B0/2 (d|k| +
    sqrt(4 + d^2 |k|^2)) in magnitude).  Returns (BlockSet at t = 0, v,
    period 1 / (|kvec| |v|))."""
    kv = np.array(kvec, np.float64)[:ndim]
    kn = float(np.linalg.norm(kv))
    K = 2 * math.pi * kn
    khat = np.zeros(3); khat[:ndim] = kv / kn
    trial = np.array([0.0, 0.0, 1.0]) if abs(khat[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(trial, khat); e1 /= np.linalg.norm(e1)
    e2 = np.cross(khat, e1)
    v = B0 * (-d * K / 2 + branch * math.sqrt(1 + (d * K / 2) ** 2))
    om = K * v
    n, dx, xlo, nbr, _ = uniform_blocks(ndim, [N] * ndim, [block or N] * ndim)

    def f(X, Y, Z):
        shape = np.broadcast_shapes(X.shape, Y.shape, Z.shape)
        xs = [X, Y, Z]
        ph = np.zeros(shape)
        for q in range(ndim):
            ph = ph + 2 * math.pi * kvec[q] * xs[q]
        b1, b2 = amp * np.cos(ph), amp * np.sin(ph)
        c = -(K * B0 / om)
        B = [B0 * khat[q] + b1 * e1[q] + b2 * e2[q] for q in range(3)]
        V = [c * (b1 * e1[q] + b2 * e2[q]) for q in range(3)]
        one = np.ones(shape)
        return {"rho": one, "p": p0 * one, "vx": V[0] * one, "vy": V[1] * one, "vz": V[2] * one,
                "Bx": B[0] * one, "By": B[1] * one, "Bz": B[2] * one}
    return sample_blocks(ndim, True, gamma, n, dx, xlo, nbr, f), v, 1.0 / (kn * abs(v))


def as_glm(bs: BlockSet, psi: float = 0.0) -> BlockSet:
    """The MHD block list `bs` as a GLM-MHD list (Sect. 4.2): the same eight
    variables and a ninth, psi, set to `psi` everywhere (ghosts included)."""
    if bs.mhd is not True and bs.mhd != 1:
        raise ValueError("as_glm needs an MHD block list")
    out = bs.copy()
    out.mhd = 2
    out.u = [np.ascontiguousarray(np.concatenate([u, np.full((1,) + u.shape[1:], psi)], axis=0))
             for u in bs.u]
    return out


def riemann_1d(left: Dict[str, float], right: Dict[str, float], N: int, mhd: bool,
               gamma: float, lo: float = 0.0, hi: float = 1.0, x0: float = 0.5,
               nblocks: int = 1) -> BlockSet:
    """Riemann problem on [lo, hi] with fixed ghost layers (non-periodic)."""
    n, dx, xlo, nbr, _ = uniform_blocks(1, [N], [N // nblocks], lo=(lo, 0, 0), hi=(hi, 1, 1),
                                        periodic=False)

    def f(X, Y, Z):
        out = {}
        for key in set(left) | set(right):
            out[key] = np.where(X < x0, left.get(key, 0.0), right.get(key, 0.0))
        return out
    return sample_blocks(1, mhd, gamma, n, dx, xlo, nbr, f)


def sod(N: int = 200, nblocks: int = 1) -> BlockSet:
    return riemann_1d({"rho": 1.0, "p": 1.0}, {"rho": 0.125, "p": 0.1}, N, False, 1.4,
                      nblocks=nblocks)


def brio_wu(N: int = 512) -> BlockSet:
    """Sect. 4.5.2 shock tube on x in [-1, 1], gamma 5/3."""
    L = {"rho": 1.0, "p": 1.0, "Bx": 0.75, "By": 1.0}
    R = {"rho": 0.125, "p": 0.1, "Bx": 0.75, "By": -1.0}
    return riemann_1d(L, R, N, True, 5.0 / 3.0, lo=-1.0, hi=1.0, x0=0.0)


def random_tangent(bs: BlockSet, seed: int, nmodes: int = 4, scale: float = 1.0,
                   vars_: Optional[Sequence[int]] = None) -> List[np.ndarray]:
    """Smooth seeded direction in state space (padded layout, ghosts zero)."""
    rng = np.random.default_rng(seed)
    out = []
    vars_ = list(range(bs.nvar)) if vars_ is None else list(vars_)
    coeffs = {v: random_modes(rng, bs.ndim, nmodes) for v in vars_}
    for b in range(bs.nb):
        X, Y, Z = cell_centres(bs.ndim, bs.n[b], bs.dx[b], bs.xlo[b])
        t = np.zeros(bs.padded_shape(b))
        for v in vars_:
            ks, a, ph = coeffs[v]
            acc = 0.0
            for k, am, p in zip(ks, a, ph):
                acc = acc + am * np.sin(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + p)
            t[v] = scale * acc / a.sum()
        inner = bs.interior(b, t).copy()
        t[...] = 0.0
        bs.interior(b, t)[...] = inner
        out.append(t)
    return out
