"""Restarted flexible GMRES with right preconditioning, FP64 (Saad's FGMRES).
Test infrastructure only.

For A x = b with a (possibly varying) preconditioner M, a cycle of m steps
builds an orthonormal Arnoldi basis v_j with z_j = M(v_j), A z_j expanded by
modified Gram-Schmidt into the Hessenberg matrix H, and sets
x = x0 + Z y with y minimising |beta e_1 - H y| (Givens rotations).  Cycles
repeat from the true residual until |b - A x| / |b| <= tol.  Each RHS is
solved independently.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class GmresStats:
    iters: int
    cycles: int
    true_rel_resid: float
    converged: bool


def _dot(a, b):
    return np.sum(a.conj() * b)


def fgmres(apply_a, b: np.ndarray, precond=None, tol: float = 1e-10, m: int = 16,
           max_cycles: int = 1000, x0=None):
    """x = A^-1 b per RHS (leading axis); precond(v) -> z, default identity."""
    precond = precond or (lambda v: v.copy())
    x = np.zeros_like(b) if x0 is None else x0.copy()
    stats = []
    for i in range(b.shape[0]):
        bi = b[i:i + 1]
        xi = x[i:i + 1]
        bnorm = np.sqrt(_dot(bi, bi).real)
        if bnorm == 0.0:
            xi[...] = 0
            stats.append(GmresStats(0, 0, 0.0, True))
            continue
        iters = cycles = 0
        converged = False
        while cycles < max_cycles:
            r = bi - apply_a(xi)
            beta = np.sqrt(_dot(r, r).real)
            if beta <= tol * bnorm:
                converged = True
                break
            cycles += 1
            v = [r / beta]
            z = []
            h = np.zeros((m + 1, m), dtype=np.complex128)
            cs = np.zeros(m, dtype=np.complex128)
            sn = np.zeros(m, dtype=np.complex128)
            g = np.zeros(m + 1, dtype=np.complex128)
            g[0] = beta
            k = 0
            for j in range(m):
                z.append(precond(v[j]))
                w = apply_a(z[j])
                for l in range(j + 1):          # modified Gram-Schmidt
                    h[l, j] = _dot(v[l], w)
                    w = w - h[l, j] * v[l]
                h[j + 1, j] = np.sqrt(_dot(w, w).real)
                v.append(w / h[j + 1, j] if h[j + 1, j] != 0 else w)
                for l in range(j):              # earlier rotations
                    t = np.conj(cs[l]) * h[l, j] + np.conj(sn[l]) * h[l + 1, j]
                    h[l + 1, j] = -sn[l] * h[l, j] + cs[l] * h[l + 1, j]
                    h[l, j] = t
                den = np.sqrt(abs(h[j, j]) ** 2 + abs(h[j + 1, j]) ** 2)
                cs[j] = h[j, j] / den
                sn[j] = h[j + 1, j] / den
                h[j, j] = den
                h[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = np.conj(cs[j]) * g[j]
                k = j + 1
                iters += 1
                if abs(g[j + 1]) <= tol * bnorm:
                    break
            y = np.linalg.solve(np.triu(h[:k, :k]), g[:k])
            for j in range(k):
                xi += y[j] * z[j]
        r = bi - apply_a(xi)
        stats.append(GmresStats(iters, cycles, float(np.sqrt(_dot(r, r).real) / bnorm), converged))
    return x, stats
