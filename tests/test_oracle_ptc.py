"""Pins of the oracle's PTC network and FGMRES (no GPU): gauge equivariance,
the free-field (unit-link) case as an ordinary convolution computed by FFT,
adjoint consistency, gradients against finite differences, and FGMRES against
scipy's GMRES and an exact-inverse preconditioner."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import synth
from oracle import fgmres, ptc
from oracle.dirac import WilsonDirac
from tests import gauge_util


def _net(dims, bc, seed=5, eps=0.5, unit=False):
    u = synth.unit_links(dims, bc) if unit else synth.random_links(dims, bc, eps, seed)
    d = WilsonDirac(dims, bc, 0.12, u)
    w1, w2 = ptc.init_weights(seed + 1, scale=0.3)
    return u, d, ptc.Transport(d), w1, w2


@pytest.mark.parametrize("bc", ["sf", "periodic", "antiperiodic"])
def test_ptc_gauge_equivariance(bc):
    dims = (4, 2, 2, 4)
    u, d, tr, w1, w2 = _net(dims, bc)
    r = synth.gaussian_spinors(dims, bc, 2, 9)
    om = synth.random_gauge_transform(dims, bc, 3002)
    dt = WilsonDirac(dims, bc, 0.12, gauge_util.rotate_links(u, om, bc))
    rot = lambda f: gauge_util.rotate_spinors(f, om, bc)
    y, _ = ptc.forward(tr, w1, w2, r)
    yt, _ = ptc.forward(ptc.Transport(dt), w1, w2, rot(r))
    np.testing.assert_allclose(yt, rot(y), atol=1e-12)


def test_ptc_free_field_is_an_fft_convolution():
    """Unit links, periodic: each layer is a 9-point stencil convolution,
    diagonal in momentum space: out(k) = sum_p W_p phase_p(k) in(k)."""
    dims = (4, 6, 2, 4)
    _, d, tr, w1, _ = _net(dims, "periodic", unit=True)
    x = synth.gaussian_spinors(dims, "periodic", 1, 11)[0]          # [t][z][y][x][4][3]
    got = ptc.layer(tr, w1, x[None, None])[:, 0]                      # [8][t][z][y][x][4][3]
    axes = (0, 3, 2, 1)                                               # array axis of mu
    xk = np.fft.fftn(x, axes=(0, 1, 2, 3))
    kgrid = np.meshgrid(*[np.fft.fftfreq(n) * 2 * np.pi for n in x.shape[:4]], indexing="ij")
    want = np.zeros((8,) + x.shape, dtype=complex)
    for co in range(8):
        acc = np.einsum("st,...ta->...sa", w1[0, co, 0], xk)
        for mu in range(4):
            k = kgrid[axes[mu]]
            # forward path: psi(n + mu) -> e^{+ik}; backward: psi(n - mu) -> e^{-ik}
            acc += np.exp(1j * k)[..., None, None] * np.einsum("st,...ta->...sa", w1[1 + mu, co, 0], xk)
            acc += np.exp(-1j * k)[..., None, None] * np.einsum("st,...ta->...sa", w1[5 + mu, co, 0], xk)
        want[co] = np.fft.ifftn(acc, axes=(0, 1, 2, 3))
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_layer_adjoint_consistency():
    dims, bc = (4, 2, 4, 4), "sf"
    _, d, tr, w1, w2 = _net(dims, bc)
    rng = np.random.default_rng(1)
    x = synth.gaussian_spinors(dims, bc, 8, 12)[:, None]              # [8 ch][1 rhs]...
    g = synth.gaussian_spinors(dims, bc, 1, 13)[None]
    lhs = np.vdot(g, ptc.layer(tr, w2, x))
    rhs = np.vdot(ptc.layer_adjoint(tr, w2, g), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    for p in range(9):
        a = synth.gaussian_spinors(dims, bc, 1, 20 + p)
        b = synth.gaussian_spinors(dims, bc, 1, 40 + p)
        assert abs(np.vdot(a, tr.apply(p, b)) - np.vdot(tr.adjoint(p, a), b)) < 1e-12 * np.abs(a).sum()
    assert rng is not None


def test_loss_gradient_matches_finite_differences():
    dims, bc = (2, 2, 2, 4), "sf"
    _, d, tr, w1, w2 = _net(dims, bc)
    r = synth.gaussian_spinors(dims, bc, 3, 14)
    e = synth.gaussian_spinors(dims, bc, 3, 15)
    loss, g1, g2 = ptc.loss_and_grad(tr, w1, w2, r, e)
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(12):
        which = int(rng.integers(2))
        w = (w1 if which == 0 else w2).copy()
        idx = tuple(int(rng.integers(n)) for n in w.shape)
        for part, unit in ((0, 1.0), (1, 1j)):
            wp, wm = w.copy(), w.copy()
            wp[idx] += h * unit
            wm[idx] -= h * unit
            args_p = (wp, w2) if which == 0 else (w1, wp)
            args_m = (wm, w2) if which == 0 else (w1, wm)
            fd = (ptc.loss_and_grad(tr, *args_p, r, e)[0] - ptc.loss_and_grad(tr, *args_m, r, e)[0]) / (2 * h)
            g = (g1 if which == 0 else g2)[idx]
            an = g.real if part == 0 else g.imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (which, idx, part, fd, an)


def test_adam_reduces_loss_on_a_fixed_pair_set():
    dims, bc = (2, 2, 2, 4), "sf"
    _, d, tr, w1, w2 = _net(dims, bc)
    r = synth.gaussian_spinors(dims, bc, 4, 16)
    e = synth.gaussian_spinors(dims, bc, 4, 17)
    m1 = v1 = m2 = v2 = 0
    first = None
    for t in range(1, 31):
        loss, g1, g2 = ptc.loss_and_grad(tr, w1, w2, r, e)
        first = loss if first is None else first
        w1, m1, v1 = ptc.adam_step(w1, g1, m1, v1, t, lr=1e-2)
        w2, m2, v2 = ptc.adam_step(w2, g2, m2, v2, t, lr=1e-2)
    assert loss < 0.8 * first


def test_fgmres_one_cycle_equals_scipy_gmres():
    dims, bc = (2, 2, 2, 4), "sf"
    d = WilsonDirac(dims, bc, 0.12, synth.random_links(dims, bc, 0.5, 3))
    a = d.dense("DdagD")
    b = synth.gaussian_spinors(dims, bc, 1, 4)
    x, st = fgmres.fgmres(d.DdagD, b, tol=1e-30, m=16, max_cycles=1)
    xs, _ = sla.gmres(a, b.reshape(-1), restart=16, maxiter=1, rtol=1e-30, atol=0)
    assert np.abs(x.reshape(-1) - xs).max() < 1e-12 * np.abs(xs).max()
    assert st[0].iters == 16


def test_fgmres_exact_inverse_converges_in_one_step_and_solves():
    dims, bc = (2, 2, 2, 4), "sf"
    d = WilsonDirac(dims, bc, 0.12, synth.random_links(dims, bc, 0.5, 3))
    a = d.dense("DdagD")
    ainv = np.linalg.inv(a)
    b = synth.gaussian_spinors(dims, bc, 2, 4)
    x, st = fgmres.fgmres(d.DdagD, b, precond=lambda v: (ainv @ v.reshape(-1)).reshape(v.shape), tol=1e-12)
    assert all(s.iters == 1 for s in st)
    x2, st2 = fgmres.fgmres(d.DdagD, b, tol=1e-12)
    want = np.linalg.solve(a, b.reshape(2, -1).T).T.reshape(b.shape)
    assert np.abs(x2 - want).max() < 1e-9 * np.abs(want).max()
    assert all(s.true_rel_resid <= 1e-12 for s in st2)


# ---- Adam (Kingma and Ba, "Adam: A method for stochastic optimization",
# Algorithm 1), each of Re and Im a real parameter of its own.

def test_adam_first_step_is_lr_times_sign_per_real_part():
    """From m = v = 0 the bias-corrected moments at t = 1 are g and g^2, so
    every real parameter moves by lr g / (|g| + eps): lr sign(g) for |g| >> eps,
    separately for Re and Im (a mixed-up Re/Im second moment would scale one
    part by the other's magnitude)."""
    g = np.array([3.0 - 0.002j, -0.5 + 7.0j, 1e-3 + 0j])
    w = np.array([0.25 + 0.5j, -1.0 + 0.0j, 2.0 - 3.0j])
    lr, eps = 0.01, 1e-8
    w1, m1, v1 = ptc.adam_step(w, g, 0, 0, 1, lr=lr, eps=eps)
    want = w - lr * (g.real / (np.abs(g.real) + eps) + 1j * g.imag / (np.abs(g.imag) + eps))
    np.testing.assert_allclose(w1, want, rtol=0, atol=1e-15)
    # 1e-3 is still >> eps: a full lr step (to 1e-5 of lr), even though |g|
    # is 3000x smaller than the largest component
    np.testing.assert_allclose((w - w1).real, lr * np.sign(g.real), atol=2e-5 * lr)
    np.testing.assert_allclose((w - w1)[:2].imag, lr * np.sign(g.imag[:2]), atol=2e-5 * lr)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * (g.real ** 2 + 1j * g.imag ** 2), rtol=1e-15)


def test_adam_two_steps_of_a_scalar_by_hand():
    """w0 = 1, lr = 0.1, g1 = 1/2, g2 = -1/4 (beta = 0.9, 0.999), worked out by
    hand in exact fractions: m1 = 1/20, v1 = 1/4000, so m^ = 1/2 and v^ = 1/4
    and w1 = 1 - 0.1 (1/2) / (1/2 + eps) = 0.900000002;
    m2 = 9/10 * 1/20 - 1/40 = 1/50, v2 = 999/1000 * 1/4000 + 1/16000
    = 1249/4000000, m^ = (1/50) / (19/100) = 2/19,
    v^ = (1249/4000000) / (1999/1000000) = 1249/7996, sqrt(v^) = 0.3952253807016642,
    w2 = w1 - 0.1 (2/19) / (0.3952253807016642 + eps) = 0.8733662987078462."""
    w, m, v = np.array([1.0 + 0j]), 0, 0
    w, m, v = ptc.adam_step(w, np.array([0.5 + 0j]), m, v, 1, lr=0.1)
    assert abs(m[0].real - 1 / 20) < 1e-15 and abs(v[0].real - 1 / 4000) < 1e-17
    assert abs(w[0].real - 0.900000002) < 1e-15
    w, m, v = ptc.adam_step(w, np.array([-0.25 + 0j]), m, v, 2, lr=0.1)
    assert abs(m[0].real - 1 / 50) < 1e-15
    assert abs(v[0].real - 1249 / 4000000) < 1e-17
    assert abs(w[0].real - 0.8733662987078462) < 1e-14
    assert w[0].imag == 0.0 and m[0].imag == 0.0 and v[0].imag == 0.0


def test_adam_bias_correction_makes_constant_gradients_exact():
    """With the same gradient every step, m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2 exactly, so the bias-corrected step is
    lr g / (|g| + eps) at every t (a wrong power in the correction, e.g.
    b^(t+1), shrinks the early steps)."""
    g = np.array([0.3 - 2.0j, -4.0 + 0.01j])
    w = np.zeros(2, dtype=complex)
    m = v = 0
    lr = 1e-3
    for t in range(1, 8):
        w_new, m, v = ptc.adam_step(w, g, m, v, t, lr=lr)
        step = w - w_new
        want = lr * (g.real / (np.abs(g.real) + 1e-8) + 1j * g.imag / (np.abs(g.imag) + 1e-8))
        np.testing.assert_allclose(step, want, rtol=1e-9)
        w = w_new
