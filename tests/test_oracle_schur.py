"""Pins of the oracle's even/odd (Schur complement) operator and of the
even/odd action variant (no GPU): the dense Schur complement of the dense D,
adjointness and gamma5-hermiticity, solves through the Schur complement
against dense solves of D and D^+, and the variant's force against finite
differences of its action."""
import numpy as np
import pytest

import synth
from oracle import force as fmod
from oracle import hmc, schur, solvers
from oracle.dirac import GAMMA5, WilsonDirac, even_odd_mask

CASES = [((2, 2, 2, 4), "sf", 0.12, 0.5), ((2, 4, 2, 4), "periodic", 0.11, 0.5),
         ((4, 2, 2, 4), "antiperiodic", 0.12, 0.3)]


def _expi(h):
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * w)) @ v.conj().T


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[1])
def test_schur_operator_is_the_dense_schur_complement(case):
    """D^ = D_ee - D_eo D_oo^-1 D_oe with the blocks taken from the dense full
    operator (coded independently of the even/odd form)."""
    dims, bc, kappa, eps = case
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, eps, 1000))
    full = d.dense("D")
    ev = np.broadcast_to(even_odd_mask(dims, bc)[..., None, None], d.spinor_shape(1)[1:]).reshape(-1)
    e, o = np.flatnonzero(ev), np.flatnonzero(~ev)
    want = full[np.ix_(e, e)] - full[np.ix_(e, o)] @ np.linalg.solve(full[np.ix_(o, o)], full[np.ix_(o, e)])
    s = schur.Schur(d)
    got, idx = s.dense()
    np.testing.assert_array_equal(idx, e)
    assert np.abs(got - want).max() < 1e-14 * np.abs(want).max()
    # the adjoint operator is the conjugate transpose, and gamma5-hermiticity holds
    gotd, _ = s.dense(dagger=True)
    assert np.abs(gotd - got.conj().T).max() < 1e-14
    g5 = np.kron(np.eye(e.size // 12), np.kron(GAMMA5, np.eye(3)))
    assert np.abs(g5 @ got @ g5 - gotd).max() < 1e-14


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[1])
def test_schur_solves_reproduce_dense_solves(case):
    dims, bc, kappa, eps = case
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, eps, 1001))
    s = schur.Schur(d)
    phi = synth.gaussian_spinors(dims, bc, 2, 2001)
    x, _ = s.solve_D(phi, 1e-14)
    want = solvers.dense_solve(d, phi, "D")
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-12
    y, _ = s.solve_D(phi, 1e-14, dagger=True)
    want = solvers.dense_solve(d, phi, "Ddag")
    assert np.linalg.norm(y - want) / np.linalg.norm(want) < 1e-12


def test_eo_action_force_matches_finite_differences():
    """The variant's force (full-lattice X, Y rebuilt from the even-site
    solutions) against 4th-order central differences of S_eo computed by a
    dense solve of D^ under U_mu(n) -> exp(i w T^a) U_mu(n)."""
    dims, bc, kappa = (2, 2, 2, 4), "sf", 0.12
    u = synth.random_links(dims, bc, 0.5, 21)
    phi = synth.gaussian_spinors(dims, bc, 2, 22)
    d = WilsonDirac(dims, bc, kappa, u)
    g, act, x, y = schur.eo_force(d, phi, dense=True)
    assert abs(np.sum(act) - schur.eo_action_dense(dims, bc, kappa, u, phi)) < 1e-12 * np.sum(act)
    fa = fmod.matrix_to_coefficients(g)
    mask = hmc.entering_mask(dims, bc)
    assert not np.any(g[~mask])
    rng = np.random.default_rng(3)
    for _ in range(8):
        mu = int(rng.integers(4))
        t = int(rng.integers(1, 4)) if mu else int(rng.integers(1, 3))
        z, yy, xx = (int(v) for v in rng.integers(2, size=3))
        a = int(rng.integers(8))

        def s_of(w):
            u2 = u.copy()
            u2[mu, t, z, yy, xx] = _expi(w * fmod.TA[a]) @ u2[mu, t, z, yy, xx]
            return schur.eo_action_dense(dims, bc, kappa, u2, phi)
        e = 1e-3
        fd = (-s_of(2 * e) + 8 * s_of(e) - 8 * s_of(-e) + s_of(-2 * e)) / (12 * e)
        assert abs(fd - fa[mu, t, z, yy, xx, a]) < 1e-8 * max(1.0, abs(fd)), (mu, t, a, fd)
    # the CG route gives the same force
    g2, act2, _, _ = schur.eo_force(d, phi, tol=1e-14)
    assert np.abs(g2 - g).max() < 1e-11 * np.abs(g).max()
    np.testing.assert_allclose(act2, act, rtol=1e-12)
    # X and Y are the full-lattice D^-1 and (D^+)^-1 images of the even-site
    # sources: D X = phi_e on the even sites and 0 on the odd ones
    s = schur.Schur(d)
    np.testing.assert_allclose(d.D(x), s.pe(phi), atol=1e-12)
    np.testing.assert_allclose(d.Ddag(y), s.pe(x), atol=1e-12)
