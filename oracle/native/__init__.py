"""The oracle's plain-C Wilson hopping term (test infrastructure only).

``NativeWilson`` has the same interface as ``oracle.dirac.WilsonDirac`` (hop,
D, Ddag, DdagD, DDdag) but runs the hopping term in a plain C loop with OpenMP
over sites, so that CG on config-sized lattices finishes in seconds.  It is
pinned against the numpy definition and against the same closed forms.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wilson_ref.c")
LIB = os.path.join(HERE, "libwilson_ref.so")
_BC = {"sf": 0, "periodic": 1, "antiperiodic": 2}
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fcx-limited-range", "-fopenmp", "-shared", "-fPIC", "-std=c11", SRC, "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        i = ctypes.c_int
        lib.wilson_ref_hop.argtypes = [p, p, p, i, i, i, i, i, i, i]
        lib.wilson_ref_hop.restype = None
        lib.wilson_ref_gamma.argtypes = [i, p]
        lib.wilson_ref_gamma.restype = None
        lib.wilson_ref_set_threads.argtypes = [i]
        lib.wilson_ref_set_threads.restype = None
        lib.wilson_ref_get_threads.argtypes = []
        lib.wilson_ref_get_threads.restype = i
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Thread count of the compiled operator (n <= 0: OpenMP's default);
    returns the count now in force."""
    lib = _load()
    lib.wilson_ref_set_threads(int(n))
    return int(lib.wilson_ref_get_threads())


def gamma(mu: int) -> np.ndarray:
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().wilson_ref_gamma(mu, out.ctypes.data)
    return out


class NativeWilson:
    def __init__(self, dims, bc, kappa, links):
        self.dims = tuple(int(d) for d in dims)
        self.bc = bc
        self.kappa = float(kappa)
        self.U = np.ascontiguousarray(links, dtype=np.complex128)
        lx, ly, lz, t = self.dims
        self.t_dyn = t - 1 if bc == "sf" else t
        want = (4, t + 1 if bc == "sf" else t, lz, ly, lx, 3, 3)
        if self.U.shape != want:
            raise ValueError(f"links shape {self.U.shape}, expected {want}")
        _load()

    def spinor_shape(self, n_rhs):
        lx, ly, lz, _ = self.dims
        return (n_rhs, self.t_dyn, lz, ly, lx, 4, 3)

    def hop(self, psi, dagger=False):
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        out = np.empty_like(psi)
        lx, ly, lz, t = self.dims
        _lib.wilson_ref_hop(self.U.ctypes.data, psi.ctypes.data, out.ctypes.data, lx, ly, lz, t,
                            _BC[self.bc], psi.shape[0], int(dagger))
        return out

    def D(self, psi):
        return psi - self.kappa * self.hop(psi)

    def Ddag(self, psi):
        return psi - self.kappa * self.hop(psi, dagger=True)

    def DdagD(self, psi):
        return self.Ddag(self.D(psi))

    def DDdag(self, psi):
        return self.D(self.Ddag(psi))
