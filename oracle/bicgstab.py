"""BiCGStab solvers of the paper's blocked algorithm, FP64.  Test
infrastructure only.

Section 3.1 solves the blocked equations D X = B (the second and third lines
of Alg. 2) with the even/odd-preconditioned Wilson operator and compares the
sequential per-RHS BiCGStab with two block forms; Section 3.2 adds a
mixed-precision preconditioner, an inner single-precision solve per RHS
called from the double-precision outer iteration.  The methods reach the plain
definition X = D^-1 B, which is what parity compares against; these
implementations exist to pin the algorithms (and to count iterations):

* ``bicgstab`` -- van der Vorst's BiCGStab per right-hand side, with an
  optional right preconditioner K (x = K^-1-side iterate).
* ``gl_bicgstab`` -- the global form: the recurrences of BiCGStab with every
  inner product replaced by the Frobenius product <X, Y> = Tr X^H Y over the
  block, so all RHS share the scalars.
* ``bl_bicgstab`` -- the block form: alpha and beta are s x s matrices from
  the shadow block R~ (the initial residuals), omega a scalar:
      V = A P^,  (R~^H V) alpha = R~^H R,  S = R - V alpha,  T = A S^,
      omega = Tr(T^H S) / Tr(T^H T),  X += P^ alpha + omega S^,
      R = S - omega T,  (R~^H V) beta = -R~^H T,  P = R + (P - omega V) beta,
  with P^ = K^-1 P and S^ = K^-1 S (identity without a preconditioner).

Blocks are arrays whose leading axis is the RHS.  Every solver stops when
every RHS's TRUE residual |b - A x| / |b| is at most tol (recomputed when the
recursion claims it), and restarts from the true residual if the recursion
lied.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class BiStats:
    iters: int
    true_rel_resid: list
    converged: bool


def _vdot(a, b):
    return np.sum(a.conj() * b)


def _cols(a):
    return a.reshape(a.shape[0], -1)


def _apply_cols(f, blk):
    return np.concatenate([f(blk[i:i + 1]) for i in range(blk.shape[0])])


def _true_res(apply_a, b, x):
    r = b - _apply_cols(apply_a, x)
    return r, [float(np.linalg.norm(r[i]) / np.linalg.norm(b[i])) if np.any(b[i]) else 0.0
                for i in range(b.shape[0])]


def _finish(apply_a, b, x, it, tol):
    _, res = _true_res(apply_a, b, x)
    return x, BiStats(it, res, all(v <= tol for v in res))


def bicgstab(apply_a, b, tol, max_iter=100000, precond=None):
    """Per-RHS BiCGStab (one column after the other, as Alg. 1 runs the
    flavours).  Returns (x, [BiStats per RHS])."""
    k_inv = precond if precond is not None else (lambda v: v.copy())
    xs, stats = [], []
    for i in range(b.shape[0]):
        bi = b[i:i + 1]
        x = np.zeros_like(bi)
        bn = np.linalg.norm(bi)
        if bn == 0.0:
            xs.append(x)
            stats.append(BiStats(0, [0.0], True))
            continue
        it = 0
        while True:
            r = bi - apply_a(x)
            if np.linalg.norm(r) <= tol * bn or it >= max_iter:
                break
            rt = r.copy()
            rho = alpha = omega = 1.0 + 0j
            v = np.zeros_like(r)
            p = np.zeros_like(r)
            while it < max_iter:
                rho_new = _vdot(rt, r)
                if rho_new == 0:
                    break
                beta = (rho_new / rho) * (alpha / omega)
                p = r + beta * (p - omega * v)
                ph = k_inv(p)
                v = apply_a(ph)
                alpha = rho_new / _vdot(rt, v)
                s = r - alpha * v
                sh = k_inv(s)
                t = apply_a(sh)
                tt = _vdot(t, t).real
                omega = _vdot(t, s) / tt if tt > 0 else 0.0
                x = x + alpha * ph + omega * sh
                r = s - omega * t
                rho = rho_new
                it += 1
                if np.linalg.norm(r) <= tol * bn or omega == 0:
                    break
        xs.append(x)
        _, res = _true_res(apply_a, bi, x)
        stats.append(BiStats(it, res, res[0] <= tol))
    return np.concatenate(xs), stats


def gl_bicgstab(apply_a, b, tol, max_iter=100000, precond=None):
    """Global BiCGStab on the whole block.  Returns (x, BiStats)."""
    k_inv = precond if precond is not None else (lambda v: v.copy())
    x = np.zeros_like(b)
    bn = np.linalg.norm(_cols(b), axis=1)
    it = 0
    while True:
        r, res = _true_res(apply_a, b, x)
        if all(v <= tol for v in res) or it >= max_iter:
            break
        rt = r.copy()
        rho = _vdot(rt, r)
        p = r.copy()
        while it < max_iter:
            ph = _apply_cols(k_inv, p)
            v = _apply_cols(apply_a, ph)
            alpha = rho / _vdot(rt, v)
            s = r - alpha * v
            sh = _apply_cols(k_inv, s)
            t = _apply_cols(apply_a, sh)
            omega = _vdot(t, s) / _vdot(t, t).real
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            it += 1
            if np.all(np.linalg.norm(_cols(r), axis=1) <= tol * bn):
                break
            rho_new = _vdot(rt, r)
            p = r + (rho_new / rho) * (alpha / omega) * (p - omega * v)
            rho = rho_new
    return _finish(apply_a, b, x, it, tol)


def bl_bicgstab(apply_a, b, tol, max_iter=100000, precond=None):
    """Block BiCGStab (s x s alpha and beta, scalar omega).  Returns (x, BiStats)."""
    k_inv = precond if precond is not None else (lambda v: v.copy())
    x = np.zeros_like(b)
    bn = np.linalg.norm(_cols(b), axis=1)
    it = 0

    def gram(a, c):  # a^H c, s x s
        return _cols(a).conj() @ _cols(c).T

    def mix(blk, m):  # column i of the result = sum_j blk_j m[j, i]
        return np.tensordot(m, blk, axes=([0], [0]))

    while True:
        r, res = _true_res(apply_a, b, x)
        if all(v <= tol for v in res) or it >= max_iter:
            break
        rt = r.copy()
        p = r.copy()
        while it < max_iter:
            ph = _apply_cols(k_inv, p)
            v = _apply_cols(apply_a, ph)
            g = gram(rt, v)
            alpha = np.linalg.solve(g, gram(rt, r))
            s = r - mix(v, alpha)
            sh = _apply_cols(k_inv, s)
            t = _apply_cols(apply_a, sh)
            omega = _vdot(t, s) / _vdot(t, t).real
            x = x + mix(ph, alpha) + omega * sh
            r = s - omega * t
            it += 1
            if np.all(np.linalg.norm(_cols(r), axis=1) <= tol * bn):
                break
            beta = np.linalg.solve(g, -gram(rt, t))
            p = r + mix(p - omega * v, beta)
    return _finish(apply_a, b, x, it, tol)
