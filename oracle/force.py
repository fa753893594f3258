"""Pseudo-fermion action and MD force, FP64.  Test infrastructure only.

Action (Eq. 2): S = sum_i |D^-1 phi_i|^2 with N_f/2 additive pseudo-fermions.

Force (Eq. 3): F_mu(n) = sum_i f[x_i, y_i] with x_i = D^-1 phi_i and
y_i = (D^+)^-1 x_i.  The paper defines f only as the derivative of
|D^-1 phi_i|^2 with respect to the gauge field.  Reading used here: perturb one
link as U_mu(n) -> exp(i w T^a) U_mu(n), T^a = lambda^a / 2, and take

    F^a_mu(n) = dS/dw^a
              = -2 sum_i Re[ y_i^+ (dD/dw^a) x_i ]
              = 2 kappa sum_i Re{ i [ y_i(n)^+ (1 - g_mu) T^a U_mu(n) x_i(n+mu)
                                      - y_i(n+mu)^+ (1 + g_mu) U_mu(n)^+ T^a x_i(n) ] }

coded literally, one generator at a time.  The stored output is the Hermitian
traceless matrix G_mu(n) = sum_a F^a_mu(n) T^a (so F^a = 2 Tr T^a G).  Links
that never enter D (the SF boundary links) get exactly zero.
"""
from __future__ import annotations

import numpy as np

from .dirac import GAMMA, ONE4, WilsonDirac
from . import solvers

# T^a = lambda^a / 2, the su(3) generators of the perturbation.
_L = np.zeros((8, 3, 3), dtype=np.complex128)
_L[0][0, 1] = _L[0][1, 0] = 1
_L[1][0, 1], _L[1][1, 0] = -1j, 1j
_L[2][0, 0], _L[2][1, 1] = 1, -1
_L[3][0, 2] = _L[3][2, 0] = 1
_L[4][0, 2], _L[4][2, 0] = -1j, 1j
_L[5][1, 2] = _L[5][2, 1] = 1
_L[6][1, 2], _L[6][2, 1] = -1j, 1j
_L[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
TA = _L / 2


def action(dirac: WilsonDirac, x: np.ndarray) -> np.ndarray:
    """Per-pseudo-fermion action S_i = |x_i|^2 with x_i = D^-1 phi_i."""
    return np.array([np.vdot(x[i], x[i]).real for i in range(x.shape[0])])


def force_coefficients(dirac: WilsonDirac, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """F^a_mu(n), shape [mu][x0][z][y][x][8], summed over the RHS axis of x, y."""
    k = dirac.kappa
    xf = dirac.embed(x)
    yf = dirac.embed(y)
    out = np.zeros(dirac.U.shape[:5] + (8,))
    for mu in range(4):
        u = dirac.U[mu]
        x_fwd = dirac.shift_fwd(xf, mu)          # x(n + mu)
        y_fwd = dirac.shift_fwd(yf, mu)          # y(n + mu)
        for a in range(8):
            t = TA[a]
            # term 1: y(n)^+ (1 - g_mu) T^a U_mu(n) x(n + mu)
            v1 = x_fwd @ np.swapaxes(t @ u, -1, -2)        # (T^a U) x, colour
            v1 = (ONE4 - GAMMA[mu]) @ v1                    # spin projector
            term1 = np.sum(yf.conj() * v1, axis=(0, 5, 6))
            # term 2: y(n + mu)^+ (1 + g_mu) U_mu(n)^+ T^a x(n)
            v2 = xf @ np.swapaxes(u.conj().swapaxes(-1, -2) @ t, -1, -2)
            v2 = (ONE4 + GAMMA[mu]) @ v2
            term2 = np.sum(y_fwd.conj() * v2, axis=(0, 5, 6))
            out[mu, ..., a] = 2.0 * k * np.real(1j * (term1 - term2))
    return out


def coefficients_to_matrix(fa: np.ndarray) -> np.ndarray:
    """G = sum_a F^a T^a (Hermitian traceless 3x3 per link)."""
    return np.einsum("...a,aij->...ij", fa, TA)


def matrix_to_coefficients(g: np.ndarray) -> np.ndarray:
    """F^a = 2 Tr(T^a G)."""
    return 2.0 * np.einsum("aij,...ji->...a", TA, g).real


def fermion_force(dirac: WilsonDirac, phi: np.ndarray, tol: float = 1e-14,
                  max_iter: int = 100000):
    """Alg. 2: X = D^-1 Phi, Y = (D^+)^-1 X, G = sum_i f[x_i, y_i], S_i.

    Returns (G [mu][x0][z][y][x][3][3], S [n_rhs], X, Y)."""
    x, _ = solvers.solve_D(dirac, phi, tol, max_iter)
    y, _ = solvers.solve_Ddag(dirac, x, tol, max_iter)
    g = coefficients_to_matrix(force_coefficients(dirac, x, y))
    return g, action(dirac, x), x, y


def fermion_force_dense(dirac: WilsonDirac, phi: np.ndarray):
    """Same as ``fermion_force`` with dense direct solves (tiny lattices)."""
    x = solvers.dense_solve(dirac, phi, "D")
    y = solvers.dense_solve(dirac, x, "Ddag")
    g = coefficients_to_matrix(force_coefficients(dirac, x, y))
    return g, action(dirac, x), x, y


def action_dense(dims, bc, kappa, links, phi) -> float:
    """S = sum_i |D^-1 phi_i|^2 by a dense solve (tiny lattices)."""
    d = WilsonDirac(dims, bc, kappa, links)
    x = solvers.dense_solve(d, phi, "D")
    return float(np.sum(np.abs(x) ** 2))
