"""MI355X many-flavor blocked quark solve.

Python face of libmfq.so (hand-written HIP for gfx950 behind a C ABI, see
``include/mfq.h``).  ``Lattice`` wraps one handle: it owns the packed links and
calls the library's Wilson hopping operator, batched multi-RHS CG on D^+D and
blocked fermion force (the paper's Alg. 2 with Eq. 2 and Eq. 3).  Tensors are
complex128 device tensors in the canonical layouts described in the header.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import BC, OPS, PREC, MfqError, SolveStats, make_params

__all__ = ["Lattice", "MfqError", "make_params", "BC", "OPS", "PREC"]


def spinor_shape(dims, bc, n_rhs):
    lx, ly, lz, t = dims
    td = t - 1 if bc == "sf" else t
    return (n_rhs, td, lz, ly, lx, 4, 3)


def link_shape(dims, bc):
    lx, ly, lz, t = dims
    ts = t + 1 if bc == "sf" else t
    return (4, ts, lz, ly, lx, 3, 3)


class Lattice:
    """One lattice (dims = (Lx, Ly, Lz, T), boundary, kappa) and its links."""

    def __init__(self, dims, bc: str, kappa: float, links: torch.Tensor, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.bc = bc
        self.kappa = float(kappa)
        if tuple(links.shape) != link_shape(self.dims, bc):
            raise ValueError(f"links shape {tuple(links.shape)} != {link_shape(self.dims, bc)}")
        lib = _lib.lib()
        lat = _lib._Lattice((ctypes.c_int * 4)(*self.dims), BC[bc], self.kappa)
        h = ctypes.c_void_p()
        _lib.check(lib.mfq_create(ctypes.byref(lat), _lib.dptr(links), _lib.stream_ptr(stream),
                                  ctypes.byref(h)))
        self._h = h

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().mfq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_links(self, links: torch.Tensor, stream=None):
        _lib.check(_lib.lib().mfq_update_links(self._h, _lib.dptr(links), _lib.stream_ptr(stream)))

    def spinor_shape(self, n_rhs: int):
        return spinor_shape(self.dims, self.bc, n_rhs)

    def _check_spinor(self, psi: torch.Tensor) -> int:
        if psi.dim() != 7 or tuple(psi.shape[1:]) != self.spinor_shape(1)[1:]:
            raise ValueError(f"spinor shape {tuple(psi.shape)} does not match the lattice")
        return int(psi.shape[0])

    # ------------------------------------------------------------------
    def dslash(self, op: str, psi: torch.Tensor, prec: str = "fp64", stream=None) -> torch.Tensor:
        n = self._check_spinor(psi)
        out = torch.empty_like(psi)
        _lib.check(_lib.lib().mfq_dslash_prec(self._h, OPS[op], PREC[prec], _lib.dptr(psi), _lib.dptr(out),
                                             n, _lib.stream_ptr(stream)))
        return out

    def solve(self, b: torch.Tensor, params=None, stream=None, **kw):
        """x = (D^+D)^-1 b for all RHS at once; returns (x, [stats dicts], status)."""
        n = self._check_spinor(b)
        p = params if params is not None else make_params(**kw)
        x = torch.empty_like(b)
        stats = (SolveStats * n)()
        rc = _lib.lib().mfq_solve_multi_rhs(self._h, _lib.dptr(b), _lib.dptr(x), n, ctypes.byref(p),
                                            stats, _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1))
        return x, [s.as_dict() for s in stats], rc

    def force(self, phi: torch.Tensor, params=None, want_xy: bool = False, stream=None, **kw):
        """Alg. 2: returns (G, action[n], stats, status[, X, Y])."""
        n = self._check_spinor(phi)
        p = params if params is not None else make_params(**kw)
        g = torch.empty(link_shape(self.dims, self.bc), dtype=torch.complex128, device=phi.device)
        action = (ctypes.c_double * n)()
        stats = (SolveStats * n)()
        x = torch.empty_like(phi) if want_xy else None
        y = torch.empty_like(phi) if want_xy else None
        rc = _lib.lib().mfq_fermion_force(
            self._h, _lib.dptr(phi), n, ctypes.byref(p), _lib.dptr(g), action,
            _lib.dptr(x) if want_xy else None, _lib.dptr(y) if want_xy else None, stats,
            _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1))
        out = (g, list(action), [s.as_dict() for s in stats], rc)
        return out + (x, y) if want_xy else out

    def time_hop(self, prec: str, n_rhs: int, iters: int = 50, stream=None) -> float:
        """Average ms of one launch of the inner solver's fused half-dslash."""
        ms = ctypes.c_double()
        _lib.check(_lib.lib().mfq_time_hop(self._h, PREC[prec], int(n_rhs), int(iters),
                                          _lib.stream_ptr(stream), ctypes.byref(ms)))
        return ms.value
