"""Leapfrog molecular dynamics with the pseudo-fermion action only, FP64.
Test infrastructure only.

The paper's HMC (Section 2) adds the pseudo-fermion action to the gauge action
and a kinetic term.  Here only the fermion part is kept (the plaquette action
is not on the path):

    H = 1/2 sum_{n,mu,a} (P^a_mu(n))^2 + sum_i |D^-1 phi_i|^2,

with dU/dt = i P U, P = sum_a P^a T^a, and dP^a/dt = -F^a (the force of
Eq. 3).  Leapfrog: P -= dt/2 F; U <- exp(i dt P) U; P -= dt/2 F.  Its energy
error at fixed trajectory length scales as dt^2.
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonDirac
from . import force as fmod
from . import solvers


def entering_mask(dims, bc) -> np.ndarray:
    """[mu][x0][z][y][x] True for links that enter D."""
    lx, ly, lz, t = dims
    ts = t + 1 if bc == "sf" else t
    m = np.ones((4, ts, lz, ly, lx), dtype=bool)
    if bc == "sf":
        m[:, 0] = False          # x0 = 0: spatial boundary links, U_0(0)
        m[1:, -1] = False        # x0 = T: spatial boundary links
        m[0, -2:] = False        # U_0(T-1) and U_0(T) never enter
    return m


def _expi(p: np.ndarray) -> np.ndarray:
    """exp(i P) for Hermitian P, batched."""
    w, v = np.linalg.eigh(p)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


class FermionMD:
    def __init__(self, dims, bc, kappa, phi, dense: bool = True, tol: float = 1e-14):
        self.dims, self.bc, self.kappa, self.phi = tuple(dims), bc, float(kappa), phi
        self.dense, self.tol = dense, tol
        self.mask = entering_mask(dims, bc)

    def _dirac(self, u):
        return WilsonDirac(self.dims, self.bc, self.kappa, u)

    def action(self, u) -> float:
        d = self._dirac(u)
        if self.dense:
            x = solvers.dense_solve(d, self.phi, "D")
        else:
            x, _ = solvers.solve_D(d, self.phi, self.tol)
        return float(np.sum(np.abs(x) ** 2))

    def force(self, u) -> np.ndarray:
        d = self._dirac(u)
        if self.dense:
            g, _, _, _ = fmod.fermion_force_dense(d, self.phi)
        else:
            g, _, _, _ = fmod.fermion_force(d, self.phi, self.tol)
        return fmod.matrix_to_coefficients(g)

    def hamiltonian(self, u, p) -> float:
        return 0.5 * float(np.sum(p[self.mask] ** 2)) + self.action(u)

    def leapfrog(self, u, p, tau: float, n_steps: int):
        dt = tau / n_steps
        u = u.copy()
        p = p * self.mask[..., None]
        p = p - 0.5 * dt * self.force(u)
        for step in range(n_steps):
            pm = fmod.coefficients_to_matrix(p)
            u = np.where(self.mask[..., None, None], _expi(dt * pm) @ u, u)
            f = self.force(u)
            p = p - (dt if step + 1 < n_steps else 0.5 * dt) * f
        return u, p

    def delta_h(self, u, p, tau: float, n_steps: int) -> float:
        p = p * self.mask[..., None]
        h0 = self.hamiltonian(u, p)
        u1, p1 = self.leapfrog(u, p, tau, n_steps)
        return self.hamiltonian(u1, p1) - h0
