"""ctypes front-end of the plain FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package.  The HIP product path never does.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

RK3, SSPRK43, SSPRK54 = 0, 1, 2
STAGES = {RK3: 3, SSPRK43: 4, SSPRK54: 5}
MP5, LIM03 = 0, 1


class OracleError(RuntimeError):
    pass


def lib():
    global _LIB
    if _LIB is None:
        # AMRVAC_ORACLE_LIB: another build of the same source (the
        # sanitizer test's)
        path = os.environ.get("AMRVAC_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401
            _b.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        dpp = ctypes.POINTER(dp)
        L.orc_mp5.restype = ctypes.c_double
        L.orc_mp5.argtypes = [dp, ctypes.c_double]
        L.orc_mp5_grad.restype = ctypes.c_double
        L.orc_mp5_grad.argtypes = [dp, ctypes.c_double, dp]
        L.orc_lim03.restype = ctypes.c_double
        L.orc_lim03.argtypes = [dp, ctypes.c_double]
        L.orc_lim03_grad.restype = ctypes.c_double
        L.orc_lim03_grad.argtypes = [dp, ctypes.c_double, dp]
        L.orc_set_lim03_radius.argtypes = [ctypes.c_double]
        L.orc_set_recon.argtypes = [ctypes.c_int]
        L.orc_prim.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_flux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_flux_glm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_set_hall.argtypes = [ctypes.c_double]
        L.orc_flux_hall.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        L.orc_glm_cr.restype = ctypes.c_double
        L.orc_set_glm_cr.argtypes = [ctypes.c_double]
        L.orc_fast_speed.restype = ctypes.c_double
        L.orc_fast_speed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp]
        L.orc_scheme_table.argtypes = [ctypes.c_int, dp, dp]
        L.orc_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, ip, dp, ip, dpp, dpp, dp, dp]
        L.orc_cmax.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ip, dp, ip,
                               dpp, dp]
        L.orc_divb.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ip, dp, ip, dpp, dpp]
        L.orc_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int, ip, dp, ip, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, dpp, dp]
        L.orc_run_jvp.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ip, dp, ip, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, dpp, dpp]
        L.orc_run_vjp.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ip, dp, ip, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, dpp, dpp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_count_ops.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, ip, dp, ip, dpp, ctypes.c_int, ctypes.c_int, u64p, u64p, u64p]
        L.orc_set_mp5_median.argtypes = [ctypes.c_int]
        L.orc_branch_hash_end.restype = ctypes.c_uint64
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_active.argtypes = [ctypes.POINTER(ctypes.c_ubyte), ctypes.c_int]
        _LIB = L
    return _LIB


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _ptrs(arrs: Sequence[np.ndarray]):
    dp = ctypes.POINTER(ctypes.c_double)
    P = (dp * len(arrs))()
    for i, a in enumerate(arrs):
        P[i] = _dp(a)
    return P


def _geom(bs):
    n = np.ascontiguousarray(bs.n, np.int32)
    dx = np.ascontiguousarray(bs.dx, np.float64)
    nbr = np.ascontiguousarray(bs.nbr, np.int32)
    return n, dx, nbr


def _check(st: int, what: str):
    if st != 0:
        raise OracleError(f"oracle {what} failed with status {st}")


def mp5(f: Sequence[float], eps: float = 0.0) -> float:
    a = np.ascontiguousarray(f, np.float64)
    return lib().orc_mp5(_dp(a), eps)


def mp5_grad(f: Sequence[float], eps: float = 0.0) -> Tuple[float, np.ndarray]:
    a = np.ascontiguousarray(f, np.float64)
    g = np.zeros(5)
    v = lib().orc_mp5_grad(_dp(a), eps, _dp(g))
    return v, g


def lim03(f: Sequence[float], dx: float = 1.0) -> float:
    """LIM03 left-biased interface value at j+1/2 from f_{j-1}, f_j, f_{j+1}
    on cells of width dx (dx scales the asymptotic-region test)."""
    a = np.ascontiguousarray(f, np.float64)
    assert a.size == 3
    return lib().orc_lim03(_dp(a), dx)


def lim03_grad(f: Sequence[float], dx: float = 1.0) -> Tuple[float, np.ndarray]:
    a = np.ascontiguousarray(f, np.float64)
    g = np.zeros(3)
    v = lib().orc_lim03_grad(_dp(a), dx, _dp(g))
    return v, g


def set_lim03_radius(r: float) -> None:
    """Radius of LIM03's asymptotic region (test hook; default 1)."""
    lib().orc_set_lim03_radius(float(r))


def set_recon(recon: int) -> None:
    """Reconstruction of the later rhs / run / run_jvp calls: MP5 (the
    default) or LIM03 (both offered in Sect. 2.2)."""
    _check(lib().orc_set_recon(int(recon)), "set_recon")


class use_recon:
    """Context manager: `with use_recon(LIM03): ...` restores MP5 on exit."""

    def __init__(self, recon: int):
        self.recon = recon

    def __enter__(self):
        set_recon(self.recon)
        return self

    def __exit__(self, *exc):
        set_recon(MP5)
        return False


def prim(ndim: int, mhd: bool, gamma: float, u: Sequence[float]) -> Tuple[int, np.ndarray]:
    a = np.zeros(9); a[:len(u)] = u
    w = np.zeros(8)
    st = lib().orc_prim(ndim, int(mhd), gamma, _dp(a), _dp(w))
    return st, w


def flux(ndim: int, mhd: bool, gamma: float, d: int, u: Sequence[float]) -> np.ndarray:
    a = np.zeros(9); a[:len(u)] = u
    f = np.zeros(9)
    lib().orc_flux(ndim, int(mhd), gamma, d, _dp(a), _dp(f))
    return f[:len(u)]


def flux_glm(ndim: int, gamma: float, d: int, ch: float, u: Sequence[float]) -> np.ndarray:
    """GLM flux (Sect. 4.2, glm3) of the 9-variable state u along d."""
    a = np.zeros(9); a[:len(u)] = u
    f = np.zeros(9)
    lib().orc_flux_glm(ndim, gamma, d, ch, _dp(a), _dp(f))
    return f


def set_hall(eta_h: float) -> None:
    """Hall parameter of the later MHD rhs / run / cmax calls (Sect. 4.4;
    0 = ideal MHD)."""
    lib().orc_set_hall(float(eta_h))


class use_hall:
    """Context manager: `with use_hall(eta_h): ...` restores ideal MHD."""

    def __init__(self, eta_h: float):
        self.eta_h = eta_h

    def __enter__(self):
        set_hall(self.eta_h)
        return self

    def __exit__(self, *exc):
        set_hall(0.0)
        return False


def flux_hall(ndim: int, gamma: float, eta_h: float, d: int, u: Sequence[float], J: Sequence[float]) -> np.ndarray:
    """MHD flux along d with the Hall terms for the current J."""
    a = np.zeros(9); a[:len(u)] = u
    j = np.ascontiguousarray(J, np.float64)
    f = np.zeros(9)
    lib().orc_flux_hall(ndim, gamma, eta_h, d, _dp(a), _dp(j), _dp(f))
    return f[:8]


def glm_cr() -> float:
    return lib().orc_glm_cr()


def set_glm_cr(cr: float) -> None:
    """Test hook: c_r of the GLM psi decay (default 0.18)."""
    lib().orc_set_glm_cr(float(cr))


def fast_speed(ndim: int, mhd: bool, gamma: float, d: int, u: Sequence[float]) -> float:
    a = np.zeros(9); a[:len(u)] = u
    return lib().orc_fast_speed(ndim, int(mhd), gamma, d, _dp(a))


def scheme_table(scheme: int):
    al = np.zeros(36); be = np.zeros(36)
    s = lib().orc_scheme_table(scheme, _dp(al), _dp(be))
    return s, al.reshape(6, 6)[:s + 1, :s], be.reshape(6, 6)[:s + 1, :s]


def rhs(bs, eps: float = 0.0, cmax: Optional[Sequence[float]] = None
        ) -> Tuple[List[np.ndarray], np.ndarray]:
    """L(U) for every block (padded arrays, ghost entries 0) and c_max[3].
    `cmax` overrides the maximum over these blocks (for samples of a larger
    block list)."""
    n, dx, nbr = _geom(bs)
    u = [np.ascontiguousarray(x, np.float64) for x in bs.u]
    out = [np.zeros_like(x) for x in u]
    cm = np.zeros(3)
    cin = None if cmax is None else np.ascontiguousarray(cmax, np.float64)
    st = lib().orc_rhs(bs.ndim, int(bs.mhd), bs.gamma, eps, bs.nb, _ip(n), _dp(dx), _ip(nbr),
                       _ptrs(u), _ptrs(out), _dp(cm), None if cin is None else _dp(cin))
    _check(st, "rhs")
    return out, (cm if cin is None else cin.copy())


def cmax(bs) -> np.ndarray:
    """Global c_max over the interior cells of every block."""
    n, dx, nbr = _geom(bs)
    u = [np.ascontiguousarray(x, np.float64) for x in bs.u]
    cm = np.zeros(3)
    st = lib().orc_cmax(bs.ndim, int(bs.mhd), bs.gamma, bs.nb, _ip(n), _dp(dx), _ip(nbr), _ptrs(u),
                        _dp(cm))
    _check(st, "cmax")
    return cm


def divb(bs) -> List[np.ndarray]:
    """div B by fourth-order central differences at every interior cell
    (Sect. 4.5.1 monitor); per block an array of the interior shape
    (nz, ny, nx)."""
    n, dx, nbr = _geom(bs)
    u = [np.ascontiguousarray(x, np.float64) for x in bs.u]
    out = [np.zeros(int(np.prod(bs.n[b]))) for b in range(bs.nb)]
    st = lib().orc_divb(bs.ndim, int(bs.mhd), bs.gamma, bs.nb, _ip(n), _dp(dx), _ip(nbr), _ptrs(u), _ptrs(out))
    _check(st, "divb")
    return [o.reshape(int(bs.n[b, 2]), int(bs.n[b, 1]), int(bs.n[b, 0])) for b, o in enumerate(out)]


def run(bs, scheme: int, nsteps: int, cfl: float = 0.4, dt: Optional[float] = None,
        eps: float = 0.0):
    """nsteps steps; returns (new BlockSet, per-step dt array)."""
    n, dx, nbr = _geom(bs)
    out = bs.copy()
    out.u = [np.ascontiguousarray(x, np.float64).copy() for x in bs.u]
    dts = np.zeros(max(nsteps, 1))
    st = lib().orc_run(bs.ndim, int(bs.mhd), bs.gamma, eps, bs.nb, _ip(n), _dp(dx), _ip(nbr),
                       scheme, cfl, -1.0 if dt is None else float(dt), nsteps, _ptrs(out.u),
                       _dp(dts))
    _check(st, "run")
    return out, dts[:nsteps]


def run_jvp(bs, tangent: Sequence[np.ndarray], scheme: int, nsteps: int, dt: float,
            eps: float = 0.0):
    """Forward-mode JVP of U0 -> U_N at fixed dt; returns (U_N BlockSet, dU_N list)."""
    n, dx, nbr = _geom(bs)
    out = bs.copy()
    out.u = [np.ascontiguousarray(x, np.float64).copy() for x in bs.u]
    du = [np.ascontiguousarray(t, np.float64).copy() for t in tangent]
    st = lib().orc_run_jvp(bs.ndim, int(bs.mhd), bs.gamma, eps, bs.nb, _ip(n), _dp(dx), _ip(nbr),
                           scheme, float(dt), nsteps, _ptrs(out.u), _ptrs(du))
    _check(st, "jvp")
    return out, du


def run_vjp(bs, lam_n: Sequence[np.ndarray], scheme: int, nsteps: int, dt: float,
            eps: float = 0.0) -> List[np.ndarray]:
    """Reverse mode of U0 -> U_N at fixed dt (local dual-number Jacobians,
    transposed and scattered): from lam_N = dJ/dU_N (padded, ghosts ignored)
    returns dJ/dU_0 (padded): interiors, plus the adjoint of the boundary data
    in the face ghosts of fixed faces; every other ghost entry is 0."""
    n, dx, nbr = _geom(bs)
    u = [np.ascontiguousarray(x, np.float64).copy() for x in bs.u]
    lam = [np.ascontiguousarray(x, np.float64).copy() for x in lam_n]
    st = lib().orc_run_vjp(bs.ndim, int(bs.mhd), bs.gamma, eps, bs.nb, _ip(n), _dp(dx), _ip(nbr),
                           scheme, float(dt), nsteps, _ptrs(u), _ptrs(lam))
    _check(st, "vjp")
    return lam


OP_CATEGORIES = ("other", "flux", "recon", "diff", "cmax", "stage")


def count_ops(bs, scheme: int = SSPRK54, median_form: bool = False, eps: float = 0.0):
    """Operation counts of one step (CFL 0.4) on the block list, single
    threaded: per category (OP_CATEGORIES) the arithmetic operations, the
    comparisons and selections, and the units they were spent on."""
    n, dx, nbr = _geom(bs)
    u = [np.ascontiguousarray(x, np.float64) for x in bs.u]
    nops = np.zeros(6, np.uint64)
    ncmp = np.zeros(6, np.uint64)
    units = np.zeros(6, np.uint64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    st = lib().orc_count_ops(bs.ndim, int(bs.mhd), bs.gamma, eps, bs.nb, _ip(n), _dp(dx), _ip(nbr), _ptrs(u),
                             scheme, int(median_form), nops.ctypes.data_as(u64p), ncmp.ctypes.data_as(u64p),
                             units.ctypes.data_as(u64p))
    _check(st, "count_ops")
    return {c: {"ops": int(a), "cmp": int(b), "units": int(k)}
            for c, a, b, k in zip(OP_CATEGORIES, nops, ncmp, units)}


class mp5_median_form:
    """Context manager: MP5 without its early exit (the median form) in the
    oracle's later calls; restored on exit."""

    def __enter__(self):
        lib().orc_set_mp5_median(1)
        return self

    def __exit__(self, *exc):
        lib().orc_set_mp5_median(0)
        return False


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def set_active(flags: Optional[Sequence[int]]) -> None:
    """Dynamic grid activation (appendix "Dynamic grid activation"): later
    calls on a block list of len(flags) blocks advance only the blocks with a
    nonzero flag; passive blocks keep their state and act as ghost sources.
    None: every block active."""
    if flags is None:
        lib().orc_set_active(None, 0)
        return
    arr = (ctypes.c_ubyte * len(flags))(*[1 if f else 0 for f in flags])
    lib().orc_set_active(arr, len(flags))


def run_branch_hash(bs, scheme: int, nsteps: int, dt: float, eps: float = 0.0) -> int:
    """Fingerprint of every branch decision of a forward run (single thread);
    equal fingerprints at U0 +/- h dU certify a non-kinked difference quotient."""
    nthreads = num_threads()
    lib().orc_branch_hash_begin()
    try:
        run(bs, scheme, nsteps, dt=dt, eps=eps)
    finally:
        h = int(lib().orc_branch_hash_end())
        set_threads(nthreads)
    return h
