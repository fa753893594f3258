"""Pins of the oracle's solvers, action, force and MD (no GPU).

Solutions are pinned to LAPACK direct solves; the force (Eq. 3) to finite
differences of the action (Eq. 2); the leapfrog to its dt^2 energy error."""
import numpy as np
import pytest

import synth
from oracle import force as fmod
from oracle import hmc, solvers
from oracle.dirac import GAMMA5, WilsonDirac
from tests import gauge_util

TINY = ((2, 2, 2, 4), "sf", 0.12)


def _expi(h):
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * w)) @ v.conj().T


@pytest.mark.parametrize("case", [((2, 2, 2, 4), "sf", 0.12, 0.5),
                                  ((4, 4, 4, 4), "sf", 0.125, 0.3),
                                  ((2, 4, 2, 4), "antiperiodic", 0.12, 0.3)])
def test_cg_matches_dense_solve(case):
    dims, bc, kappa, eps = case
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, eps, 1000))
    b = synth.gaussian_spinors(dims, bc, 2, 2000)
    x, stats = solvers.cg_normal(d, b, 1e-13)
    want = solvers.dense_solve(d, b, "DdagD")
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-11
    for s in stats:
        assert s.converged and s.true_rel_resid <= 1e-13
    xd, _ = solvers.solve_D(d, b, 1e-13)
    assert np.linalg.norm(xd - solvers.dense_solve(d, b, "D")) / np.linalg.norm(xd) < 1e-11
    yd, _ = solvers.solve_Ddag(d, b, 1e-13)
    assert np.linalg.norm(yd - solvers.dense_solve(d, b, "Ddag")) / np.linalg.norm(yd) < 1e-11


def test_cg_zero_rhs_and_max_iter():
    dims, bc, kappa = TINY
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, 0.5, 1))
    b = synth.gaussian_spinors(dims, bc, 2, 2)
    b[1] = 0
    x, st = solvers.cg_normal(d, b, 1e-12, max_iter=3)
    assert not st[0].converged and st[0].iters == 3
    assert st[1].converged and st[1].iters == 0 and not np.any(x[1])


def test_lanczos_condition_estimate():
    dims, bc, kappa = (2, 2, 2, 6), "sf", 0.13
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, 0.5, 3))
    ev = np.linalg.eigvalsh(d.dense("DdagD"))
    b = synth.gaussian_spinors(dims, bc, 1, 4)
    est = solvers.cg_cond(d.DdagD, b, 120)
    assert abs(est / (ev[-1] / ev[0]) - 1) < 1e-3


def test_force_matches_finite_differences():
    dims, bc, kappa = TINY
    u = synth.random_links(dims, bc, 0.5, 11)
    phi = synth.gaussian_spinors(dims, bc, 2, 12)
    d = WilsonDirac(dims, bc, kappa, u)
    g, s, _, _ = fmod.fermion_force_dense(d, phi)
    fa = fmod.matrix_to_coefficients(g)
    assert abs(np.sum(s) - fmod.action_dense(dims, bc, kappa, u, phi)) < 1e-12 * np.sum(s)
    rng = np.random.default_rng(0)
    for _ in range(8):
        mu = int(rng.integers(4))
        t = int(rng.integers(1, 4)) if mu else int(rng.integers(1, 3))
        z, y, x = (int(v) for v in rng.integers(2, size=3))
        a = int(rng.integers(8))

        def s_of(w):
            u2 = u.copy()
            u2[mu, t, z, y, x] = _expi(w * fmod.TA[a]) @ u2[mu, t, z, y, x]
            return fmod.action_dense(dims, bc, kappa, u2, phi)
        e = 1e-3
        fd = (-s_of(2 * e) + 8 * s_of(e) - 8 * s_of(-e) + s_of(-2 * e)) / (12 * e)
        assert abs(fd - fa[mu, t, z, y, x, a]) < 1e-8 * max(1.0, abs(fd))


def test_force_random_directional_derivative():
    """d/dw S(exp(i w X) U) at w = 0 equals sum_links F^a X^a for a global
    random direction X."""
    dims, bc, kappa = (2, 2, 4, 4), "periodic", 0.11
    u = synth.random_links(dims, bc, 0.5, 31)
    phi = synth.gaussian_spinors(dims, bc, 1, 32)
    d = WilsonDirac(dims, bc, kappa, u)
    g, _, _, _ = fmod.fermion_force_dense(d, phi)
    fa = fmod.matrix_to_coefficients(g)
    xa = np.random.default_rng(5).standard_normal(fa.shape)
    xm = fmod.coefficients_to_matrix(xa)

    def s_of(w):
        w_, v = np.linalg.eigh(w * xm)
        ex = np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w_), v.conj())
        return fmod.action_dense(dims, bc, kappa, ex @ u, phi)
    e = 1e-3
    fd = (-s_of(2 * e) + 8 * s_of(e) - 8 * s_of(-e) + s_of(-2 * e)) / (12 * e)
    assert abs(fd - np.sum(fa * xa)) < 1e-8 * abs(fd)


def test_force_invariants():
    """Hermitian traceless output, zero on links that never enter D, gauge
    covariance, and linearity over pseudo-fermion shards."""
    dims, bc, kappa = (2, 4, 2, 4), "sf", 0.12
    u = synth.random_links(dims, bc, 0.5, 41)
    phi = synth.gaussian_spinors(dims, bc, 3, 42)
    d = WilsonDirac(dims, bc, kappa, u)
    g, s, x, y = fmod.fermion_force_dense(d, phi)
    np.testing.assert_allclose(g, np.swapaxes(g.conj(), -1, -2), atol=1e-14)
    assert np.abs(np.trace(g, axis1=-2, axis2=-1)).max() < 1e-13
    mask = hmc.entering_mask(dims, bc)
    assert not np.any(g[~mask])
    assert np.abs(g[mask]).max() > 1e-3
    # gauge covariance: G[U^Om, Om phi] = Om G[U, phi] Om^+
    om = synth.random_gauge_transform(dims, bc, 3001)
    dt = WilsonDirac(dims, bc, kappa, gauge_util.rotate_links(u, om, bc))
    gt, st, _, _ = fmod.fermion_force_dense(dt, gauge_util.rotate_spinors(phi, om, bc))
    np.testing.assert_allclose(gt, gauge_util.rotate_link_field(g, om), atol=1e-12)
    np.testing.assert_allclose(st, s, rtol=1e-12)
    # linearity: the sum of the forces of RHS shards is the whole force
    g1, _, _, _ = fmod.fermion_force_dense(d, phi[:1])
    g2, _, _, _ = fmod.fermion_force_dense(d, phi[1:])
    np.testing.assert_allclose(g1 + g2, g, atol=1e-12)


def test_gamma5_route_equals_two_solves():
    """Y = (D D^+)^-1 phi = g5 (D^+D)^-1 g5 phi and X = D^+ Y: one normal-
    equation solve gives both fields of Alg. 2."""
    dims, bc, kappa = (4, 4, 4, 4), "sf", 0.125
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, 0.3, 1000))
    phi = synth.gaussian_spinors(dims, bc, 1, 2000)
    x = solvers.dense_solve(d, phi, "D")
    y = solvers.dense_solve(d, x, "Ddag")
    z = solvers.dense_solve(d, GAMMA5 @ phi, "DdagD")
    np.testing.assert_allclose(GAMMA5 @ z, y, atol=1e-11)
    np.testing.assert_allclose(d.Ddag(GAMMA5 @ z), x, atol=1e-11)


def test_force_cg_route_matches_dense():
    dims, bc, kappa = (4, 4, 4, 4), "sf", 0.125
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, 0.3, 1000))
    phi = synth.gaussian_spinors(dims, bc, 1, 2000)
    g, s, _, _ = fmod.fermion_force(d, phi, tol=1e-14)
    gd, sd, _, _ = fmod.fermion_force_dense(d, phi)
    assert np.linalg.norm(g - gd) / np.linalg.norm(gd) < 1e-11
    np.testing.assert_allclose(s, sd, rtol=1e-12)


def test_delta_h_scales_as_dt_squared_and_reversible():
    dims, bc, kappa = TINY
    u = synth.random_links(dims, bc, 0.3, 11)
    phi = synth.gaussian_spinors(dims, bc, 2, 12)
    p = synth.gaussian_momenta(dims, bc, 4000)
    md = hmc.FermionMD(dims, bc, kappa, phi)
    dh = [md.delta_h(u, p, 0.5, n) for n in (4, 8, 16)]
    assert 3.5 <= dh[0] / dh[1] <= 4.5
    assert 3.5 <= dh[1] / dh[2] <= 4.5
    u1, p1 = md.leapfrog(u, p, 0.5, 8)
    u2, p2 = md.leapfrog(u1, -p1, 0.5, 8)
    assert np.abs(u2 - u).max() < 1e-12
