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

__all__ = ["Lattice", "Batch", "MfqError", "make_params", "BC", "OPS", "PREC"]


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

    def dslash_noalloc(self, op: str, psi: torch.Tensor, out: torch.Tensor = None, stream=None) -> torch.Tensor:
        """FP64 op(psi) through the entry point that allocates no device memory
        (the caller may pass the output tensor too)."""
        n = self._check_spinor(psi)
        if out is None:
            out = torch.empty_like(psi)
        elif out.shape != psi.shape or out.dtype != psi.dtype:
            raise ValueError("out must match psi")
        _lib.check(_lib.lib().mfq_dslash_noalloc(self._h, OPS[op], _lib.dptr(psi), _lib.dptr(out), n,
                                                _lib.stream_ptr(stream)))
        return out

    def solve(self, b: torch.Tensor, params=None, stream=None, **kw):
        """x = (D^+D)^-1 b for all RHS at once; returns (x, [stats dicts], status).

        Keyword arguments go to make_params: tol, max_iter, prec ("fp64", "fp32",
        "fp16"), reliable_delta, precond ("none": batched CG; "blockcg": block CG,
        FP64, at most 8 RHS; "ptc" / "identity": FGMRES with / without the learned
        preconditioner), restart, check_every, use_graph, route ("full": CG on
        D^+D; "schur": two even/odd-preconditioned solves)."""
        n = self._check_spinor(b)
        p = params if params is not None else make_params(**kw)
        x = torch.empty_like(b)
        stats = (SolveStats * n)()
        rc = _lib.lib().mfq_solve_multi_rhs(self._h, _lib.dptr(b), _lib.dptr(x), n, ctypes.byref(p),
                                            stats, _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1, 2))
        return x, [s.as_dict() for s in stats], rc

    def solve_dirac(self, b: torch.Tensor, dagger: bool = False, params=None, stream=None, **kw):
        """x = D^-1 b (or (D^+)^-1 b) through the even/odd Schur complement: CG
        on the even normal equations (precond "none") or the paper's BiCGStab
        solvers (precond "bicgstab", "gl_bicgstab", "bl_bicgstab"; prec "fp32"
        adds the FP32 inner solve as preconditioner).  Returns (x, stats, status)."""
        n = self._check_spinor(b)
        p = params if params is not None else make_params(**kw)
        x = torch.empty_like(b)
        stats = (SolveStats * n)()
        rc = _lib.lib().mfq_solve_dirac(self._h, int(bool(dagger)), _lib.dptr(b), _lib.dptr(x), n, ctypes.byref(p),
                                        stats, _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1, 2))
        return x, [s.as_dict() for s in stats], rc

    def force(self, phi: torch.Tensor, params=None, want_xy: bool = False, stream=None, eo_action=False, **kw):
        """Alg. 2: returns (G, action[n], stats, status[, X, Y]).  route="schur"
        runs its two solves through the even/odd Schur complement; eo_action=True
        evaluates the even/odd-preconditioned action |D^-1 phi_e|^2 instead."""
        n = self._check_spinor(phi)
        p = params if params is not None else make_params(**kw)
        g = torch.empty(link_shape(self.dims, self.bc), dtype=torch.complex128, device=phi.device)
        action = (ctypes.c_double * n)()
        stats = (SolveStats * n)()
        x = torch.empty_like(phi) if want_xy else None
        y = torch.empty_like(phi) if want_xy else None
        fn = _lib.lib().mfq_fermion_force_eo if eo_action else _lib.lib().mfq_fermion_force
        rc = fn(
            self._h, _lib.dptr(phi), n, ctypes.byref(p), _lib.dptr(g), action,
            _lib.dptr(x) if want_xy else None, _lib.dptr(y) if want_xy else None, stats,
            _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1, 2))
        out = (g, list(action), [s.as_dict() for s in stats], rc)
        return out + (x, y) if want_xy else out

    # ---------------------------------------------------------- molecular dynamics
    def _check_links(self, t: torch.Tensor):
        if tuple(t.shape) != link_shape(self.dims, self.bc):
            raise ValueError(f"expected links shape {link_shape(self.dims, self.bc)}, got {tuple(t.shape)}")

    def kinetic_energy(self, mom: torch.Tensor, stream=None) -> float:
        """1/2 sum P^a P^a over the links that enter D (FP64, on the GPU)."""
        self._check_links(mom)
        out = ctypes.c_double()
        _lib.check(_lib.lib().mfq_kinetic_energy(self._h, _lib.dptr(mom), ctypes.byref(out), _lib.stream_ptr(stream)))
        return out.value

    def md_momenta(self, force: torch.Tensor, mom: torch.Tensor, eps: float, stream=None):
        """mom -= eps * force on the links that enter D (in place)."""
        self._check_links(force)
        self._check_links(mom)
        _lib.check(_lib.lib().mfq_md_momenta(self._h, _lib.dptr(force), _lib.dptr(mom), float(eps),
                                            _lib.stream_ptr(stream)))

    def md_links(self, mom: torch.Tensor, links: torch.Tensor, eps: float, stream=None):
        """links <- exp(i eps P) links on the links that enter D (in place), and
        the handle's packed links refreshed."""
        self._check_links(mom)
        self._check_links(links)
        _lib.check(_lib.lib().mfq_md_links(self._h, _lib.dptr(mom), _lib.dptr(links), float(eps),
                                          _lib.stream_ptr(stream)))

    def hmc_trajectory(self, links: torch.Tensor, mom: torch.Tensor, phi: torch.Tensor, tau: float, n_steps: int,
                       rand_uniform: float, params=None, stream=None, **kw):
        """One leapfrog trajectory with Metropolis (links and mom updated in place,
        restored on rejection); returns (result dict, status).  Solve keywords as
        for solve()."""
        self._check_links(links)
        self._check_links(mom)
        n = self._check_spinor(phi)
        p = params if params is not None else make_params(**kw)
        hp = _lib.HmcParams(float(tau), int(n_steps), float(rand_uniform))
        res = _lib.HmcResult()
        rc = _lib.lib().mfq_hmc_trajectory(self._h, _lib.dptr(links), _lib.dptr(mom), _lib.dptr(phi), n,
                                           ctypes.byref(hp), ctypes.byref(p), ctypes.byref(res),
                                           _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1, 2))
        return res.as_dict(), rc

    def set_autotune(self, on: bool):
        _lib.check(_lib.lib().mfq_set_autotune(self._h, int(bool(on))))

    def hop_shape(self, prec: str, n_rhs: int):
        """(sites per workgroup, RHS per workgroup, order flags (bit 0 XCD
        remap, bit 1 z-blocked order, bit 2 LDS link tile), time-sweep length,
        direction split) of the inner solver's hopping kernel."""
        out = (ctypes.c_int * 5)()
        _lib.check(_lib.lib().mfq_hop_shape(self._h, PREC[prec], int(n_rhs), out))
        return tuple(out)

    def time_hop(self, prec: str, n_rhs: int, iters: int = 50, stream=None) -> float:
        """Average ms of one launch of the inner solver's fused half-dslash."""
        ms = ctypes.c_double()
        _lib.check(_lib.lib().mfq_time_hop(self._h, PREC[prec], int(n_rhs), int(iters),
                                          _lib.stream_ptr(stream), ctypes.byref(ms)))
        return ms.value


class Batch:
    """Many lattices (each a ``Lattice`` with its own RHS count) solved together:
    one persistent launch per CG phase for the whole batch."""

    def __init__(self, lattices, n_rhs, prec: str = "fp32", stream=None):
        self.lattices = list(lattices)
        self.n_rhs = [int(n) for n in n_rhs]
        self.prec = prec
        n = len(self.lattices)
        hs = (ctypes.c_void_p * n)(*[lat._h for lat in self.lattices])
        nr = (ctypes.c_int * n)(*self.n_rhs)
        b = ctypes.c_void_p()
        _lib.check(_lib.lib().mfq_batch_create(hs, n, nr, PREC[prec], _lib.stream_ptr(stream), ctypes.byref(b)))
        self._b = b

    @property
    def grid(self) -> int:
        return _lib.lib().mfq_batch_grid(self._b)

    @property
    def split(self) -> int:
        return _lib.lib().mfq_batch_split(self._b)

    def set_shape(self, grid: int, split: int):
        """Force the persistent grid size and the direction split of the
        inner hopping phases (otherwise chosen by the batch's tuning)."""
        _lib.check(_lib.lib().mfq_batch_set_shape(self._b, int(grid), int(split)))

    def solve(self, bs, params=None, stream=None, **kw):
        """bs: list of canonical spinor tensors; returns (xs, stats per lattice, status)."""
        if len(bs) != len(self.lattices):
            raise ValueError("one right-hand-side tensor per lattice")
        kw.setdefault("prec", self.prec)
        p = params if params is not None else make_params(**kw)
        for lat, b, n in zip(self.lattices, bs, self.n_rhs):
            if lat._check_spinor(b) != n:
                raise ValueError("RHS count differs from the batch's")
        xs = [torch.empty_like(b) for b in bs]
        n = len(bs)
        bp = (ctypes.c_void_p * n)(*[_lib.dptr(b).value for b in bs])
        xp = (ctypes.c_void_p * n)(*[_lib.dptr(x).value for x in xs])
        stats = (SolveStats * sum(self.n_rhs))()
        rc = _lib.lib().mfq_batch_solve(self._b, bp, xp, ctypes.byref(p), stats, _lib.stream_ptr(stream))
        _lib.check(rc, allow=(0, 1))
        flat = [s.as_dict() for s in stats]
        out, k = [], 0
        for nr in self.n_rhs:
            out.append(flat[k:k + nr])
            k += nr
        return xs, out, rc

    def close(self):
        if getattr(self, "_b", None):
            _lib.lib().mfq_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned preconditioner
N_PTC_COMPLEX = 2 * 9 * 8 * 16


def _w_to_array(w):
    import numpy as np
    w = np.ascontiguousarray(np.asarray(w, dtype=np.complex128).reshape(-1))
    if w.size != N_PTC_COMPLEX:
        raise ValueError(f"expected {N_PTC_COMPLEX} complex weights")
    return w


def _precond_init(self, seed: int = 0, scale: float = 0.1):
    _lib.check(_lib.lib().mfq_precond_init(self._h, int(seed), float(scale)))


def _precond_set_weights(self, w):
    a = _w_to_array(w)
    _lib.check(_lib.lib().mfq_precond_set_weights(self._h, ctypes.c_void_p(a.ctypes.data)))


def _precond_get_weights(self, which: str = "master"):
    import numpy as np
    out = np.zeros(N_PTC_COMPLEX, dtype=np.complex128)
    code = {"master": 0, "inference": 1, "adam_m": 2, "adam_v": 3}[which]
    _lib.check(_lib.lib().mfq_precond_get_weights(self._h, code, ctypes.c_void_p(out.ctypes.data)))
    return out


def _precond_apply(self, psi: torch.Tensor, stream=None) -> torch.Tensor:
    n = self._check_spinor(psi)
    out = torch.empty_like(psi)
    _lib.check(_lib.lib().mfq_precond_apply(self._h, _lib.dptr(psi), _lib.dptr(out), n, _lib.stream_ptr(stream)))
    return out


def _precond_loss_grad(self, r: torch.Tensor, e: torch.Tensor, stream=None):
    import numpy as np
    n = self._check_spinor(r)
    loss = ctypes.c_double()
    grad = np.zeros(N_PTC_COMPLEX, dtype=np.complex128)
    _lib.check(_lib.lib().mfq_precond_loss_grad(self._h, _lib.dptr(r), _lib.dptr(e), n, ctypes.byref(loss),
                                                ctypes.c_void_p(grad.ctypes.data), _lib.stream_ptr(stream)))
    return loss.value, grad


def _precond_train(self, r: torch.Tensor, e: torch.Tensor, steps: int = 100, lr: float = 1e-3, stream=None):
    import numpy as np
    n = self._check_spinor(r)
    hist = np.zeros(int(steps))
    _lib.check(_lib.lib().mfq_precond_train(self._h, _lib.dptr(r), _lib.dptr(e), n, int(steps), float(lr),
                                            ctypes.c_void_p(hist.ctypes.data), _lib.stream_ptr(stream)))
    return hist


def _precond_pairs(self, xi: torch.Tensor, every: int, n_snap: int, stream=None):
    """(r, e) training pairs from plain CG on b = A xi with the known solution
    xi, at k = every * j iterations for j = 0..n_snap-1: n_snap * n_rhs spinors each."""
    n = self._check_spinor(xi)
    shape = self.spinor_shape(n * n_snap)
    r = torch.empty(shape, dtype=torch.complex128, device=xi.device)
    e = torch.empty(shape, dtype=torch.complex128, device=xi.device)
    _lib.check(_lib.lib().mfq_precond_pairs(self._h, _lib.dptr(xi), n, int(every), int(n_snap), _lib.dptr(r),
                                            _lib.dptr(e), _lib.stream_ptr(stream)))
    return r, e


def _precond_save(self, path: str):
    _lib.check(_lib.lib().mfq_precond_save(self._h, str(path).encode()))


def _precond_load(self, path: str):
    _lib.check(_lib.lib().mfq_precond_load(self._h, str(path).encode()))


Lattice.precond_init = _precond_init
Lattice.precond_set_weights = _precond_set_weights
Lattice.precond_get_weights = _precond_get_weights
Lattice.precond_apply = _precond_apply
Lattice.precond_loss_grad = _precond_loss_grad
Lattice.precond_train = _precond_train
Lattice.precond_pairs = _precond_pairs
Lattice.precond_save = _precond_save
Lattice.precond_load = _precond_load
