"""Even/odd (Schur complement) form of the Wilson operator, FP64, full-lattice
arrays.  Test infrastructure only.

The paper preconditions its solvers by site even/odd decomposition (Section
3.1, and the GPU solver of Section 3.2) without writing the reduced operator
out.  With sites ordered (even, odd), D = 1 - kappa H has unit diagonal
blocks and off-diagonal blocks -kappa H_eo, -kappa H_oe, so its Schur
complement on the even sites is

    D^ = 1 - kappa^2 H_eo H_oe,        D^+ = 1 - kappa^2 (H^+)_eo (H^+)_oe,

and D x = phi is solved by

    D^ x_e = phi_e + kappa H_eo phi_o,      x_o = phi_o + kappa H_oe x_e.

Even-site fields are stored as full dynamical-site arrays that are zero on the
odd sites.  The even/odd-preconditioned action variant is
S_eo = sum_i |D^-1 phi_i,e|^2 with phi on the even sites; its force is the
derivative of that definition.
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonDirac, even_odd_mask
from . import force as fmod
from . import solvers


class Schur:
    """D^ and D^+ of one WilsonDirac (numpy or compiled oracle operator)."""

    def __init__(self, dirac, dims=None, bc=None):
        self.d = dirac
        dims = dims if dims is not None else dirac.dims
        bc = bc if bc is not None else dirac.bc
        self.even = even_odd_mask(dims, bc)[None, ..., None, None]
        self.kappa = dirac.kappa

    def pe(self, f):
        """Projection on the even sites."""
        return np.where(self.even, f, 0)

    def po(self, f):
        return np.where(self.even, 0, f)

    def h_eo(self, f, dagger=False):
        """(H_eo f_o) on the even sites (H^+ for dagger)."""
        return self.pe(self.d.hop(self.po(f), dagger=dagger))

    def h_oe(self, f, dagger=False):
        return self.po(self.d.hop(self.pe(f), dagger=dagger))

    def apply(self, f, dagger=False):
        """D^ f_e (or D^+ f_e); the odd part of f is ignored, the result is zero there."""
        fe = self.pe(f)
        return fe - self.kappa ** 2 * self.h_eo(self.h_oe(fe, dagger), dagger)

    def normal(self, f):
        """D^+ D^ f_e."""
        return self.apply(self.apply(f), dagger=True)

    # ---- solves through the Schur complement -------------------------------
    def solve_D(self, phi, tol, max_iter=100000, dagger=False):
        """x = D^-1 phi (or (D^+)^-1 phi) by CG on D^+D^ (or D^ D^+) for the
        even sites and the odd-site reconstruction."""
        k = self.kappa
        be = self.pe(phi) + k * self.h_eo(phi, dagger)
        if not dagger:
            xe, st = solvers.cg(self.normal, self.apply(be, dagger=True), tol, max_iter)
        else:
            xe, st = solvers.cg(lambda f: self.apply(self.apply(f, dagger=True)), self.apply(be), tol, max_iter)
        xe = self.pe(xe)
        return xe + self.po(phi) + k * self.h_oe(xe, dagger), st

    def dense(self, dagger=False):
        """The dense even-even block matrix of D^ (tiny lattices)."""
        idx = np.flatnonzero(np.broadcast_to(self.even, self.d.spinor_shape(1)).reshape(-1))
        n = int(np.prod(self.d.spinor_shape(1)))
        m = np.zeros((idx.size, idx.size), dtype=np.complex128)
        for j, col in enumerate(idx):
            e = np.zeros(n, dtype=np.complex128)
            e[col] = 1.0
            m[:, j] = self.apply(e.reshape(self.d.spinor_shape(1)), dagger).reshape(-1)[idx]
        return m, idx


def eo_action_dense(dims, bc, kappa, links, phi) -> float:
    """S_eo = sum_i |D^-1 phi_i,e|^2 by a dense solve of D^ (tiny lattices)."""
    s = Schur(WilsonDirac(dims, bc, kappa, links))
    m, idx = s.dense()
    b = s.pe(phi).reshape(phi.shape[0], -1)[:, idx]
    x = np.linalg.solve(m, b.T).T
    return float(np.sum(np.abs(x) ** 2))


def eo_force(dirac: WilsonDirac, phi, tol=1e-14, dense=False):
    """Force and action of the even/odd action variant.

    X_e = D^-1 phi_e, Y_e = (D^+)^-1 X_e; with X_o = kappa H_oe X_e and
    Y_o = kappa (H^+)_oe Y_e the variation of S_eo is 2 kappa Re[Y^+ dH X]
    (dH connects the parities only), which is what the force of Eq. 3 computes
    from full-lattice X and Y.  Returns (G, S_eo per RHS, X, Y)."""
    s = Schur(dirac)
    phie = s.pe(phi)
    if dense:
        m, idx = s.dense()
        md, _ = s.dense(dagger=True)
        n = phi.shape[0]
        b = phie.reshape(n, -1)[:, idx]
        xe_v = np.linalg.solve(m, b.T)
        ye_v = np.linalg.solve(md, xe_v)
        xe = np.zeros((n, phie[0].size), dtype=np.complex128)
        ye = np.zeros_like(xe)
        xe[:, idx] = xe_v.T
        ye[:, idx] = ye_v.T
        xe, ye = xe.reshape(phi.shape), ye.reshape(phi.shape)
    else:
        xe, _ = solvers.cg(s.normal, s.apply(phie, dagger=True), tol)
        xe = s.pe(xe)
        ye, _ = solvers.cg(lambda f: s.apply(s.apply(f, dagger=True)), s.apply(xe), tol)
        ye = s.pe(ye)
    k = dirac.kappa
    x = xe + k * s.h_oe(xe)
    y = ye + k * s.h_oe(ye, dagger=True)
    g = fmod.coefficients_to_matrix(fmod.force_coefficients(dirac, x, y))
    act = np.array([np.vdot(xe[i], xe[i]).real for i in range(phi.shape[0])])
    return g, act, x, y
