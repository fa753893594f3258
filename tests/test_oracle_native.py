"""Pins of the oracle's plain-C hopping term: it must equal the numpy
definition and satisfy the same algebra and closed forms on its own."""
import numpy as np
import pytest

import synth
from oracle import native, solvers
from oracle.dirac import GAMMA, WilsonDirac
from tests import gauge_util

CASES = [((4, 4, 4, 4), "sf"), ((6, 2, 4, 6), "periodic"), ((4, 6, 2, 4), "antiperiodic"),
         ((2, 2, 2, 4), "sf"), ((8, 8, 8, 8), "sf")]


def test_gamma_matches_numpy_basis():
    for mu in range(4):
        np.testing.assert_array_equal(native.gamma(mu), GAMMA[mu])


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}")
def test_native_hop_equals_numpy_definition(case):
    dims, bc = case
    u = synth.random_links(dims, bc, 0.5, 3)
    d = WilsonDirac(dims, bc, 0.13, u)
    n = native.NativeWilson(dims, bc, 0.13, u)
    b = synth.gaussian_spinors(dims, bc, 3, 4)
    for dag in (False, True):
        np.testing.assert_allclose(n.hop(b, dag), d.hop(b, dag), atol=1e-13)


@pytest.mark.parametrize("bc", ["sf", "periodic", "antiperiodic"])
def test_native_adjoint_and_covariance(bc):
    dims = (4, 2, 4, 4)
    u = synth.random_links(dims, bc, 0.5, 21)
    n = native.NativeWilson(dims, bc, 0.12, u)
    a = synth.gaussian_spinors(dims, bc, 1, 8)
    b = synth.gaussian_spinors(dims, bc, 1, 9)
    lhs, rhs = np.vdot(a, n.D(b)), np.vdot(n.Ddag(a), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    om = synth.random_gauge_transform(dims, bc, 3000)
    nt = native.NativeWilson(dims, bc, 0.12, gauge_util.rotate_links(u, om, bc))
    rot = lambda f: gauge_util.rotate_spinors(f, om, bc)
    np.testing.assert_allclose(nt.D(rot(b)), rot(n.D(b)), atol=1e-13)


def test_native_free_field_plane_wave():
    dims, bc, kappa = (4, 6, 2, 8), "antiperiodic", 0.11
    n = native.NativeWilson(dims, bc, kappa, synth.unit_links(dims, bc))
    lx, ly, lz, t = dims
    p = [2 * np.pi * 1.5 / t, 2 * np.pi * 2 / lx, 2 * np.pi * 1 / ly, 2 * np.pi * 1 / lz]
    x0 = np.arange(t)[:, None, None, None]
    z = np.arange(lz)[None, :, None, None]
    y = np.arange(ly)[None, None, :, None]
    x = np.arange(lx)[None, None, None, :]
    ph = np.exp(1j * (p[0] * x0 + p[1] * x + p[2] * y + p[3] * z))
    u = np.random.default_rng(1).standard_normal((4, 3)) + 0j
    psi = (ph[..., None, None] * u)[None]
    m = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) + 2j * kappa * sum(
        GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    np.testing.assert_allclose(n.D(psi), np.einsum("st,...ta->...sa", m, psi), atol=1e-13)


def test_native_cg_matches_dense():
    dims, bc, kappa = (4, 4, 4, 4), "sf", 0.125
    u = synth.random_links(dims, bc, 0.3, 1000)
    n = native.NativeWilson(dims, bc, kappa, u)
    b = synth.gaussian_spinors(dims, bc, 1, 2000)
    x, _ = solvers.cg_normal(n, b, 1e-13)
    want = solvers.dense_solve(WilsonDirac(dims, bc, kappa, u), b, "DdagD")
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-11
