"""Solvers of the FP64 oracle.  Test infrastructure only.

* ``cg`` -- Hestenes-Stiefel conjugate gradients for a Hermitian positive
  definite operator A, run independently for every right-hand side (RHS) in
  the order of Alg. 1 (one flavor after the other).  Each RHS stops on its
  own TRUE relative residual |b - A x| / |b| <= tol, recomputed when the
  recursive residual says it has converged; iteration continues from the true
  residual if the recursion lied.
* ``solve_D`` / ``solve_Ddag`` -- the two solves of Alg. 2, D X = Phi and
  D^+ Y = X, each as CG on its normal equations (D^+D X = D^+ Phi and
  D D^+ Y = D X).
* ``dense_solve`` -- direct LU solve with the dense operator (tiny lattices).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class CGStats:
    iters: int
    true_rel_resid: float
    converged: bool
    history: list


def _dot(a, b):
    # elementwise product and sum (no threaded BLAS call: it contends with the
    # OpenMP threads of the native operator)
    return np.sum(a.conj() * b)


def cg(apply_a, b: np.ndarray, tol: float, max_iter: int = 100000, x0=None):
    """x = A^-1 b per RHS.  b has the RHS as its leading axis."""
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    stats = []
    for i in range(b.shape[0]):
        bi = b[i:i + 1]
        xi = x[i:i + 1]
        bnorm = np.sqrt(_dot(bi, bi).real)
        if bnorm == 0.0:
            xi[...] = 0.0
            stats.append(CGStats(0, 0.0, True, []))
            continue
        r = bi - apply_a(xi)
        p = r.copy()
        rho = _dot(r, r).real
        hist = [np.sqrt(rho) / bnorm]
        it = 0
        converged = False
        while it < max_iter:
            if np.sqrt(rho) <= tol * bnorm:
                r_true = bi - apply_a(xi)
                rho_true = _dot(r_true, r_true).real
                if np.sqrt(rho_true) <= tol * bnorm:
                    converged = True
                    break
                r = r_true            # the recursion lied: restart from truth
                p = r.copy()
                rho = rho_true
            ap = apply_a(p)
            alpha = rho / _dot(p, ap).real
            xi += alpha * p
            r -= alpha * ap
            rho_new = _dot(r, r).real
            p = r + (rho_new / rho) * p
            rho = rho_new
            it += 1
            hist.append(np.sqrt(rho) / bnorm)
        r_true = bi - apply_a(xi)
        stats.append(CGStats(it, float(np.sqrt(_dot(r_true, r_true).real) / bnorm),
                             converged, hist))
    return x, stats


def cg_normal(dirac, b, tol, max_iter=100000):
    """x = (D^+ D)^-1 b per RHS."""
    return cg(dirac.DdagD, b, tol, max_iter)


def solve_D(dirac, phi, tol, max_iter=100000):
    """X = D^-1 Phi (Alg. 2, second line) via CG on D^+ D X = D^+ Phi."""
    return cg(dirac.DdagD, dirac.Ddag(phi), tol, max_iter)


def solve_Ddag(dirac, x, tol, max_iter=100000):
    """Y = (D^+)^-1 X (Alg. 2, third line) via CG on D D^+ Y = D X."""
    return cg(dirac.DDdag, dirac.D(x), tol, max_iter)


def dense_solve(dirac, b, op: str = "D"):
    """Direct solve op^-1 b per RHS with the dense matrix of ``op``."""
    m = dirac.dense(op)
    shape = b.shape
    flat = b.reshape(shape[0], -1).T
    return np.linalg.solve(m, flat).T.reshape(shape)


def lanczos_condition(history_alphas_betas) -> float:
    """Condition estimate of A from CG's Lanczos tridiagonal (see ``cg_cond``)."""
    alphas, betas = history_alphas_betas
    k = len(alphas)
    t = np.zeros((k, k))
    for j in range(k):
        t[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            t[j, j + 1] = t[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    w = np.linalg.eigvalsh(t)
    return float(w[-1] / w[0])


def cg_cond(apply_a, b: np.ndarray, n_iter: int) -> float:
    """Run n_iter CG steps on the first RHS and return the Lanczos estimate of
    cond(A) (ratio of extreme Ritz values)."""
    r = b[:1].copy()
    p = r.copy()
    x = np.zeros_like(r)
    rho = _dot(r, r).real
    alphas, betas = [], []
    for _ in range(n_iter):
        ap = apply_a(p)
        alpha = rho / _dot(p, ap).real
        x += alpha * p
        r -= alpha * ap
        rho_new = _dot(r, r).real
        beta = rho_new / rho
        alphas.append(alpha)
        betas.append(beta)
        p = r + beta * p
        rho = rho_new
    return lanczos_condition((alphas, betas))
