"""Python binding of the C ABI in include/amrvac.h (argument marshalling only).

Torch tensors serve as device memory and torch's current HIP stream as the
stream; every step of the scheme runs in the native library.  Importing this
module does not touch the GPU; the library is loaded on first use and a
missing or unloadable library raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamrvac.so")

OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_NONPHYSICAL, ERR_UNSUPPORTED = range(6)
HD, MHD, GLM = 0, 1, 2
RK3, SSPRK43, SSPRK54 = 0, 1, 2
EXEC_PER_BLOCK, EXEC_BATCHED, EXEC_BATCHED_SINGLE = 0, 1, 2
MP5, LIM03 = 0, 1
NGHOST = 3
ABI_VERSION = 5
NOALLOC_MAX_DOUBLES = 8388608
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "NONPHYSICAL", 5: "UNSUPPORTED"}

# Entry points declared in include/amrvac.h.
SYMBOLS = ["amrvac_abi_version", "amrvac_create", "amrvac_set_blocks", "amrvac_validate_blocks",
           "amrvac_set_exec", "amrvac_num_variants", "amrvac_variant_name", "amrvac_set_variant",
           "amrvac_get_variant",
           "amrvac_autotune", "amrvac_fd_rhs", "amrvac_divb", "amrvac_ssprk_step", "amrvac_ssprk_step_noalloc",
           "amrvac_ssprk_adjoint",
           "amrvac_activation_flags", "amrvac_set_active",
           "amrvac_sync", "amrvac_last_error", "amrvac_destroy"]


def physics_of(mhd) -> int:
    """Physics code from a BlockSet's `mhd` field: False/0 hydro, True/1
    MHD, 2 GLM-MHD."""
    return GLM if (mhd == 2) else (MHD if mhd else HD)


class AmrvacError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"amrvac: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("physics", ctypes.c_int), ("gamma", ctypes.c_double),
                ("exec", ctypes.c_int), ("recon", ctypes.c_int), ("eta_h", ctypes.c_double)]


class Block(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("xlo", ctypes.c_double * 3), ("nbr", ctypes.c_int * 6)]


_LIB = None


def lib():
    """Load libamrvac.so (raises if it is missing: there is no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"native library {LIB_PATH} is missing; build it with "
                               "`python -m paper_1407_2052_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.amrvac_abi_version.restype = ctypes.c_int
        L.amrvac_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
        L.amrvac_set_blocks.argtypes = [vp, ctypes.POINTER(Block), ip]
        L.amrvac_validate_blocks.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(Block), ip,
                                             ctypes.c_char_p, ip]
        L.amrvac_set_exec.argtypes = [vp, ip]
        L.amrvac_num_variants.argtypes = [vp]
        L.amrvac_num_variants.restype = ctypes.c_int
        L.amrvac_variant_name.argtypes = [vp, ip]
        L.amrvac_variant_name.restype = ctypes.c_char_p
        L.amrvac_set_variant.argtypes = [vp, ip]
        L.amrvac_get_variant.argtypes = [vp]
        L.amrvac_get_variant.restype = ctypes.c_int
        L.amrvac_autotune.argtypes = [vp, ip, ip, dp]
        L.amrvac_fd_rhs.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p), dp]
        L.amrvac_divb.argtypes = [vp, ctypes.POINTER(ctypes.c_void_p), dp]
        L.amrvac_ssprk_step.argtypes = [vp, ip, ctypes.c_double, dp, ip, dp]
        L.amrvac_ssprk_step_noalloc.argtypes = [vp, ip, ctypes.c_double, dp, ip, dp]
        L.amrvac_ssprk_adjoint.argtypes = [vp, ip, ctypes.c_double, ip, ip, ctypes.POINTER(ctypes.c_void_p)]
        ub = ctypes.POINTER(ctypes.c_ubyte)
        L.amrvac_activation_flags.argtypes = [ctypes.POINTER(Block), ip, ub, ip, ub]
        L.amrvac_activation_flags.restype = ctypes.c_int
        L.amrvac_set_active.argtypes = [vp, ub]
        L.amrvac_sync.argtypes = [vp]
        L.amrvac_last_error.restype = ctypes.c_char_p
        L.amrvac_last_error.argtypes = [vp]
        L.amrvac_destroy.argtypes = [vp]
        for name in ("amrvac_create", "amrvac_set_blocks", "amrvac_validate_blocks", "amrvac_set_exec",
                     "amrvac_set_variant", "amrvac_autotune",
                     "amrvac_fd_rhs", "amrvac_ssprk_step", "amrvac_ssprk_step_noalloc", "amrvac_ssprk_adjoint",
                     "amrvac_set_active",
                     "amrvac_sync"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def make_blocks(ptrs: Sequence[int], n, dx, xlo, nbr) -> ctypes.Array:
    nb = len(ptrs)
    arr = (Block * nb)()
    for b in range(nb):
        arr[b].u = ptrs[b]
        for d in range(3):
            arr[b].n[d] = int(n[b][d])
            arr[b].dx[d] = float(dx[b][d])
            arr[b].xlo[d] = float(xlo[b][d])
        for f in range(6):
            arr[b].nbr[f] = int(nbr[b][f])
    return arr


def activation_flags(nbr, want, safety: int) -> Tuple[int, np.ndarray]:
    """Active/passive flags after the safety belt (host only, no device):
    returns (number of active blocks or -1, flags)."""
    nb = len(want)
    arr = make_blocks([0] * nb, np.ones((nb, 3)), np.ones((nb, 3)), np.zeros((nb, 3)), nbr)
    w = (ctypes.c_ubyte * nb)(*[1 if x else 0 for x in want])
    out = (ctypes.c_ubyte * nb)()
    n = lib().amrvac_activation_flags(arr, nb, w, int(safety), out)
    return n, np.array(list(out), dtype=np.uint8)


def validate_blocks(ndim: int, mhd: bool, gamma: float, ptrs, n, dx, xlo, nbr,
                    recon: int = MP5) -> Tuple[int, str]:
    """Host-only validation (no device needed)."""
    cfg = Config(ndim, physics_of(mhd), gamma, EXEC_BATCHED, recon)
    arr = make_blocks(ptrs, n, dx, xlo, nbr) if len(ptrs) else None
    buf = ctypes.create_string_buffer(256)
    st = lib().amrvac_validate_blocks(ctypes.byref(cfg), arr, len(ptrs), buf, 256)
    return st, buf.value.decode()


class Context:
    """One amrvac context bound to torch's current HIP stream."""

    def __init__(self, ndim: int, mhd: bool, gamma: float, exec: int = EXEC_BATCHED, stream=None,
                 recon: int = MP5, eta_h: float = 0.0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("amrvac.Context needs a HIP device")
        self._torch = torch
        self.ndim, self.mhd, self.gamma, self.recon = ndim, bool(mhd), float(gamma), int(recon)
        self.physics = physics_of(mhd)
        self.nvar = {HD: 2 + ndim, MHD: 8, GLM: 9}[self.physics]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = Config(ndim, self.physics, gamma, exec, recon, eta_h)
        h = ctypes.c_void_p()
        st = lib().amrvac_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if st != OK:
            raise AmrvacError(st, lib().amrvac_last_error(None).decode())
        self._h = h
        self.blocks: List = []
        self.n = None

    # -- helpers ---------------------------------------------------------
    def _check(self, st: int):
        if st != OK:
            raise AmrvacError(st, lib().amrvac_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().amrvac_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -------------------------------------------------------------
    def set_blocks(self, states: Sequence, n, dx, xlo, nbr):
        """states: float64 device tensors in the padded block layout."""
        t = self._torch
        for s in states:
            if s.dtype != t.float64 or not s.is_cuda or not s.is_contiguous():
                raise ValueError("block states must be contiguous float64 device tensors")
        self.blocks = list(states)
        self.n = np.asarray(n, np.int64)
        arr = make_blocks([s.data_ptr() for s in states], n, dx, xlo, nbr)
        self._check(lib().amrvac_set_blocks(self._h, arr, len(states)))

    def set_exec(self, exec: int):
        self._check(lib().amrvac_set_exec(self._h, exec))

    def variants(self) -> List[str]:
        n = lib().amrvac_num_variants(self._h)
        return [lib().amrvac_variant_name(self._h, i).decode() for i in range(n)]

    def set_active(self, active=None):
        """Advance only the blocks with active[b] != 0 (None: every block)."""
        if active is None:
            self._check(lib().amrvac_set_active(self._h, None))
            return
        a = (ctypes.c_ubyte * len(active))(*[1 if x else 0 for x in active])
        self._check(lib().amrvac_set_active(self._h, a))

    def set_variant(self, i: int):
        self._check(lib().amrvac_set_variant(self._h, i))

    def autotune(self, scheme: int = SSPRK54, nsteps: int = 2) -> Tuple[str, List[float]]:
        n = lib().amrvac_num_variants(self._h)
        ms = (ctypes.c_double * n)()
        self._check(lib().amrvac_autotune(self._h, scheme, nsteps, ms))
        return self.current_variant(), list(ms)

    def current_variant(self) -> str:
        return lib().amrvac_variant_name(self._h, lib().amrvac_get_variant(self._h)).decode()

    def fd_rhs(self, out: Optional[Sequence] = None, want_cmax: bool = True):
        t = self._torch
        if out is None:
            out = [t.empty((self.nvar, int(nn[2]), int(nn[1]), int(nn[0])), dtype=t.float64,
                           device=self.blocks[0].device) for nn in self.n]
        ptrs = (ctypes.c_void_p * len(out))(*[o.data_ptr() for o in out])
        cm = (ctypes.c_double * 3)()
        self._check(lib().amrvac_fd_rhs(self._h, ptrs, cm if want_cmax else None))
        return out, (np.array(cm[:]) if want_cmax else None)

    def divb(self, want_field: bool = True):
        """div B (fourth-order central differences) per block as device
        tensors (nz, ny, nx), and the mean of |div B| (synchronising)."""
        t = self._torch
        out = None
        ptrs = None
        if want_field:
            out = [t.empty((int(nn[2]), int(nn[1]), int(nn[0])), dtype=t.float64, device=self.blocks[0].device)
                   for nn in self.n]
            ptrs = (ctypes.c_void_p * len(out))(*[o.data_ptr() for o in out])
        mean = ctypes.c_double(0.0)
        self._check(lib().amrvac_divb(self._h, ptrs, ctypes.byref(mean)))
        return out, mean.value

    def ssprk_step(self, scheme: int, nsteps: int, cfl: float = 0.4, dt: Optional[float] = None,
                   t: Optional[float] = 0.0) -> Optional[float]:
        """Advance nsteps; returns the end time (synchronising) unless t is None."""
        dtp = ctypes.byref(ctypes.c_double(dt)) if dt is not None else None
        tt = ctypes.c_double(t) if t is not None else None
        self._check(lib().amrvac_ssprk_step(self._h, scheme, cfl, dtp, nsteps,
                                            ctypes.byref(tt) if tt is not None else None))
        return tt.value if tt is not None else None

    def ssprk_step_noalloc(self, scheme: int, nsteps: int, cfl: float = 0.4, dt: Optional[float] = None,
                           t: Optional[float] = 0.0) -> Optional[float]:
        """ssprk_step with the stage buffers in the library's fixed device
        array (amrvac_ssprk_step_noalloc: the call allocates nothing)."""
        dtp = ctypes.byref(ctypes.c_double(dt)) if dt is not None else None
        tt = ctypes.c_double(t) if t is not None else None
        self._check(lib().amrvac_ssprk_step_noalloc(self._h, scheme, cfl, dtp, nsteps,
                                                    ctypes.byref(tt) if tt is not None else None))
        return tt.value if tt is not None else None

    def ssprk_adjoint(self, scheme: int, dt: float, nsteps: int, ckpt_every: int, lam: Sequence):
        ptrs = (ctypes.c_void_p * len(lam))(*[x.data_ptr() for x in lam])
        self._check(lib().amrvac_ssprk_adjoint(self._h, scheme, dt, nsteps, ckpt_every, ptrs))
        return lam

    def sync(self):
        self._check(lib().amrvac_sync(self._h))


def device_blocks(bs, device="cuda"):
    """Copy a BlockSet's states into one contiguous device allocation and
    return per-block views (contiguous, padded layout)."""
    import torch
    sizes = [u.size for u in bs.u]
    flat = torch.empty(sum(sizes), dtype=torch.float64, device=device)
    host = torch.from_numpy(np.concatenate([u.ravel() for u in bs.u]))
    flat.copy_(host)
    views, off = [], 0
    for u, s in zip(bs.u, sizes):
        views.append(flat[off:off + s].view(*u.shape))
        off += s
    return flat, views


def context_for(bs, exec: int = EXEC_BATCHED, device="cuda", recon: int = MP5, eta_h: float = 0.0):
    """Context + device copy of a BlockSet (returns ctx, flat, views)."""
    flat, views = device_blocks(bs, device)
    ctx = Context(bs.ndim, bs.mhd, bs.gamma, exec, recon=recon, eta_h=eta_h)
    ctx.set_blocks(views, bs.n, bs.dx, bs.xlo, bs.nbr)
    return ctx, flat, views
