"""Pins of the oracle's Wilson-Dirac operator against algebra, closed forms
and invariants (no GPU).  The paper prints no field values, so every pin here
is a mathematical fact the operator must satisfy."""
import itertools

import numpy as np
import pytest

import synth
from tests import gauge_util
from oracle.dirac import GAMMA, GAMMA5, WilsonDirac, even_odd_mask

BCS = ["sf", "periodic", "antiperiodic"]


def test_clifford_algebra_and_gamma5():
    for m, n in itertools.product(range(4), range(4)):
        anti = GAMMA[m] @ GAMMA[n] + GAMMA[n] @ GAMMA[m]
        np.testing.assert_allclose(anti, 2.0 * np.eye(4) * (m == n), atol=1e-15)
    for m in range(4):
        np.testing.assert_allclose(GAMMA[m], GAMMA[m].conj().T, atol=0)
        np.testing.assert_allclose(GAMMA5 @ GAMMA[m], -GAMMA[m] @ GAMMA5, atol=1e-15)
    np.testing.assert_allclose(GAMMA5, np.diag([1, 1, -1, -1]), atol=1e-15)


@pytest.mark.parametrize("bc", BCS)
def test_adjoint_and_gamma5_hermiticity(bc):
    dims = (4, 4, 2, 6)
    d = WilsonDirac(dims, bc, 0.13, synth.random_links(dims, bc, 0.5, 7))
    a = synth.gaussian_spinors(dims, bc, 2, 8)
    b = synth.gaussian_spinors(dims, bc, 2, 9)
    # D^+ is coded from its own formula: it must be the adjoint of D ...
    lhs = np.vdot(a, d.D(b))
    rhs = np.vdot(d.Ddag(a), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # ... and equal gamma5 D gamma5 (the relation det D = det D^+ rests on)
    g5dg5 = d.gamma5(d.D(d.gamma5(b)))
    err = np.linalg.norm(d.Ddag(b) - g5dg5) / np.linalg.norm(g5dg5)
    assert err <= 1e-15


def _plane_wave(dims, bc, k, u):
    lx, ly, lz, t = dims
    t0, td = (1, t - 1) if bc == "sf" else (0, t)
    shift = 0.5 if bc == "antiperiodic" else 0.0
    p = [2 * np.pi * (k[0] + shift) / t, 2 * np.pi * k[1] / lx,
         2 * np.pi * k[2] / ly, 2 * np.pi * k[3] / lz]
    x0 = np.arange(t0, t0 + td)[:, None, None, None]
    z = np.arange(lz)[None, :, None, None]
    y = np.arange(ly)[None, None, :, None]
    x = np.arange(lx)[None, None, None, :]
    ph = np.exp(1j * (p[0] * x0 + p[1] * x + p[2] * y + p[3] * z))
    psi = ph[None, ..., None, None] * u[None, None, None, None, None]
    return psi, p


@pytest.mark.parametrize("bc", ["periodic", "antiperiodic"])
def test_free_field_plane_waves(bc):
    """With unit links D acts on e^{ipn} u as 1 - 2k sum cos p + 2ik sum g sin p."""
    dims = (4, 6, 2, 8)
    kappa = 0.11
    d = WilsonDirac(dims, bc, kappa, synth.unit_links(dims, bc))
    rng = np.random.default_rng(3)
    for k in [(0, 0, 0, 0), (1, 2, 1, 0), (3, 5, 0, 1), (7, 1, 1, 1)]:
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, p = _plane_wave(dims, bc, k, u)
        m = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) \
            + 2j * kappa * sum(GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
        want = np.einsum("st,...ta->...sa", m, psi)
        np.testing.assert_allclose(d.D(psi), want, atol=1e-13)


def test_free_field_DdagD_spectrum_periodic():
    dims, kappa = (4, 2, 2, 4), 0.12
    d = WilsonDirac(dims, "periodic", kappa, synth.unit_links(dims, "periodic"))
    ev = np.sort(np.linalg.eigvalsh(d.dense("DdagD")))
    want = []
    lx, ly, lz, t = dims
    for k0, k1, k2, k3 in itertools.product(range(t), range(lx), range(ly), range(lz)):
        p = [2 * np.pi * k0 / t, 2 * np.pi * k1 / lx, 2 * np.pi * k2 / ly, 2 * np.pi * k3 / lz]
        lam = (1 - 2 * kappa * sum(np.cos(p))) ** 2 + 4 * kappa ** 2 * sum(np.sin(p) ** 2)
        want += [lam] * 12
    np.testing.assert_allclose(ev, np.sort(want), atol=1e-12)


def test_free_field_DdagD_spectrum_sf():
    """SF free field: the full-lattice spectrum equals the union over spatial
    momenta of time-only 4(T-1) x 4(T-1) Dirichlet problems (x 3 colours)."""
    dims, kappa = (2, 4, 2, 6), 0.125
    lx, ly, lz, t = dims
    d = WilsonDirac(dims, "sf", kappa, synth.unit_links(dims, "sf"))
    ev = np.sort(np.linalg.eigvalsh(d.dense("DdagD")))
    n = t - 1
    want = []
    one = np.eye(4)
    for k1, k2, k3 in itertools.product(range(lx), range(ly), range(lz)):
        ps = [2 * np.pi * k1 / lx, 2 * np.pi * k2 / ly, 2 * np.pi * k3 / lz]
        diag = (1 - 2 * kappa * sum(np.cos(ps))) * one \
            + 2j * kappa * sum(GAMMA[k + 1] * np.sin(ps[k]) for k in range(3))
        m = np.zeros((4 * n, 4 * n), dtype=complex)
        for i in range(n):
            m[4 * i:4 * i + 4, 4 * i:4 * i + 4] = diag
            if i + 1 < n:
                m[4 * i:4 * i + 4, 4 * i + 4:4 * i + 8] = -kappa * (one - GAMMA[0])
                m[4 * i + 4:4 * i + 8, 4 * i:4 * i + 4] = -kappa * (one + GAMMA[0])
        want += list(np.linalg.eigvalsh(m.conj().T @ m)) * 3
    np.testing.assert_allclose(ev, np.sort(want), atol=1e-12)
    assert ev[0] > 1e-3          # the SF gap keeps D nonsingular at kappa = 1/8


@pytest.mark.parametrize("bc", BCS)
def test_gauge_covariance(bc):
    """D[U^Om] Om psi = Om D[U] psi: pins link direction and daggers."""
    dims = (4, 2, 4, 4)
    u = synth.random_links(dims, bc, 0.5, 21)
    om = synth.random_gauge_transform(dims, bc, 3000)
    psi = synth.gaussian_spinors(dims, bc, 2, 22)
    d = WilsonDirac(dims, bc, 0.13, u)
    dt = WilsonDirac(dims, bc, 0.13, gauge_util.rotate_links(u, om, bc))
    rot = lambda f: gauge_util.rotate_spinors(f, om, bc)
    np.testing.assert_allclose(dt.D(rot(psi)), rot(d.D(psi)), atol=1e-13)
    np.testing.assert_allclose(dt.Ddag(rot(psi)), rot(d.Ddag(psi)), atol=1e-13)


def test_even_odd_balance():
    for dims, bc in [((4, 4, 4, 4), "sf"), ((8, 8, 8, 8), "sf"), ((4, 2, 2, 6), "periodic")]:
        m = even_odd_mask(dims, bc)
        assert m.sum() * 2 == m.size
