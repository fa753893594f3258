"""Gauge-covariant parallel-transport convolution (PTC) network, FP64.
Test infrastructure only.

The learned preconditioner is not in the paper (its flexible preconditioner is
a single-precision inner solve, Section 3.2); the architecture below is this
build's reading:

* paths p = 0..8: p = 0 is the identity, p = 1 + mu transports from the
  forward neighbour, (T_p psi)(n) = U_mu(n) psi(n + mu), and p = 5 + mu from
  the backward neighbour, (T_p psi)(n) = U_mu(n - mu)^+ psi(n - mu); the time
  boundary rules are those of the Wilson operator (zero across SF boundaries,
  sign -1 across the antiperiodic wrap);
* a layer maps channels c to c':  psi'[c'](n) = sum_c sum_p W[p, c', c] (T_p psi[c])(n),
  with W[p, c', c] a complex 4x4 matrix acting on spin (identity on colour);
* the network is two linear layers, 1 -> 8 -> 1 channels, no bias, so it is
  a fixed linear map M = L2 L1 (a valid right preconditioner for GMRES);
* training pairs (r, e): residuals r_k = b - A x_k of plain CG iterates and
  errors e_k = x* - x_k; loss = mean_k |M r_k - e_k|^2 / |e_k|^2.

Fields with channels are arrays [channel][rhs][t][z][y][x][4][3].
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonDirac

N_PATHS = 9
HIDDEN = 8


def path_mu(p: int):
    """(mu, forward?) of path p >= 1."""
    return (p - 1, True) if p <= 4 else (p - 5, False)


class Transport:
    """T_p on one gauge field (shares the oracle's boundary-aware shifts)."""

    def __init__(self, dirac: WilsonDirac):
        self.d = dirac

    def apply(self, p: int, psi: np.ndarray) -> np.ndarray:
        if p == 0:
            return psi.copy()
        d = self.d
        mu, fwd = path_mu(p)
        f = d.embed(psi)
        if fwd:
            out = d.u_times(mu, d.shift_fwd(f, mu))
        else:
            out = d.shift_bwd(d.udag_times(mu, f), mu)
        return d.restrict(out)

    def adjoint(self, p: int, psi: np.ndarray) -> np.ndarray:
        """T_p^+ : the forward transport's adjoint is the backward one."""
        if p == 0:
            return psi.copy()
        mu, fwd = path_mu(p)
        return self.apply(5 + mu if fwd else 1 + mu, psi)


def spin(w: np.ndarray, f: np.ndarray) -> np.ndarray:
    """w (4x4) acting on the spin index of f [...][4][3]."""
    return np.einsum("st,...ta->...sa", w, f)


def layer(tr: Transport, w: np.ndarray, x: np.ndarray) -> np.ndarray:
    """w: [9][C_out][C_in][4][4]; x: [C_in][rhs]...; returns [C_out][rhs]..."""
    c_out, c_in = w.shape[1], w.shape[2]
    out = np.zeros((c_out,) + x.shape[1:], dtype=np.complex128)
    for c in range(c_in):
        for p in range(N_PATHS):
            tx = tr.apply(p, x[c])
            for co in range(c_out):
                out[co] += spin(w[p, co, c], tx)
    return out


def layer_adjoint(tr: Transport, w: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Adjoint of ``layer`` in its input: [C_out][rhs]... -> [C_in][rhs]..."""
    c_out, c_in = w.shape[1], w.shape[2]
    out = np.zeros((c_in,) + g.shape[1:], dtype=np.complex128)
    for c in range(c_in):
        for p in range(N_PATHS):
            acc = np.zeros(g.shape[1:], dtype=np.complex128)
            for co in range(c_out):
                acc += spin(w[p, co, c].conj().T, g[co])
            out[c] += tr.adjoint(p, acc)
    return out


def layer_weight_grad(tr: Transport, x: np.ndarray, g: np.ndarray, c_out: int) -> np.ndarray:
    """dL/dW for a real loss L with dL/d(out) = g (as d/dRe + i d/dIm):
    G[p, c', c] = sum_{sites, colours} g[c'] (T_p x[c])^+ over spin."""
    c_in = x.shape[0]
    grad = np.zeros((N_PATHS, c_out, c_in, 4, 4), dtype=np.complex128)
    for c in range(c_in):
        for p in range(N_PATHS):
            tx = tr.apply(p, x[c])
            for co in range(c_out):
                grad[p, co, c] = np.einsum("nsa,nta->st", g[co].reshape(-1, 4, 3),
                                           tx.conj().reshape(-1, 4, 3))
    return grad


def init_weights(seed: int, hidden: int = HIDDEN, scale: float = 0.1):
    """Small random weights; the identity path of each layer starts near a
    scaled identity so that the untrained net is close to a multiple of 1."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale / np.sqrt(2)
    w1 = draw((N_PATHS, hidden, 1, 4, 4))
    w2 = draw((N_PATHS, 1, hidden, 4, 4))
    w1[0, :, 0] += np.eye(4) / np.sqrt(hidden)
    w2[0, 0, :] += np.eye(4) / np.sqrt(hidden)
    return w1, w2


def forward(tr: Transport, w1, w2, r: np.ndarray):
    """N(r) for r [rhs]...; returns (out [rhs]..., hidden [8][rhs]...)."""
    h = layer(tr, w1, r[None])
    return layer(tr, w2, h)[0], h


def loss_and_grad(tr: Transport, w1, w2, r: np.ndarray, e: np.ndarray):
    """Mean over the pairs (rhs axis) of |N(r_k) - e_k|^2 / |e_k|^2 and its
    gradients with respect to w1 and w2."""
    n = r.shape[0]
    y, h = forward(tr, w1, w2, r)
    en = np.array([np.vdot(e[k], e[k]).real for k in range(n)])
    diff = y - e
    loss = float(np.mean([np.vdot(diff[k], diff[k]).real / en[k] for k in range(n)]))
    gy = 2.0 * diff / (n * en)[:, None, None, None, None, None, None]
    g2 = layer_weight_grad(tr, h, gy[None], 1)
    gh = layer_adjoint(tr, w2, gy[None])
    g1 = layer_weight_grad(tr, r[None], gh, w1.shape[1])
    return loss, g1, g2


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update on complex weights, treating Re and Im as separate
    real parameters (g = dL/dRe + i dL/dIm)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * (g.real ** 2 + 1j * g.imag ** 2)
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    step = mh.real / (np.sqrt(vh.real) + eps) + 1j * mh.imag / (np.sqrt(vh.imag) + eps)
    return w - lr * step, m, v
