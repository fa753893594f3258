"""Pins of the oracle's BiCGStab solvers (no GPU): converged solutions of the
full and the even/odd-preconditioned Wilson operator against LAPACK solves,
one iteration with the exact inverse as preconditioner, and the block and
global forms reducing to plain BiCGStab for a single right-hand side."""
import numpy as np
import pytest

import synth
from oracle import bicgstab as bi
from oracle import schur, solvers
from oracle.dirac import WilsonDirac

CASES = [((2, 2, 2, 4), "sf", 0.12, 0.5), ((2, 4, 2, 4), "periodic", 0.11, 0.5),
         ((4, 2, 2, 4), "antiperiodic", 0.12, 0.3)]
SOLVERS = {"plain": lambda a, b, tol, **kw: bi.bicgstab(a, b, tol, **kw),
           "global": lambda a, b, tol, **kw: bi.gl_bicgstab(a, b, tol, **kw),
           "block": lambda a, b, tol, **kw: bi.bl_bicgstab(a, b, tol, **kw)}


def _ok(stats):
    return all(s.converged for s in stats) if isinstance(stats, list) else stats.converged


@pytest.mark.parametrize("kind", list(SOLVERS))
@pytest.mark.parametrize("case", CASES, ids=lambda c: c[1])
def test_bicgstab_solutions_match_dense_solves(case, kind):
    dims, bc, kappa, eps = case
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, eps, 1200))
    b = synth.gaussian_spinors(dims, bc, 3, 2200)
    # the full operator D and its adjoint
    for op, fn in (("D", d.D), ("Ddag", d.Ddag)):
        x, st = SOLVERS[kind](fn, b, 1e-13)
        assert _ok(st)
        want = solvers.dense_solve(d, b, op)
        assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-11, (op, kind)
    # the even/odd-preconditioned operator on even-site sources
    s = schur.Schur(d)
    be = s.pe(b)
    x, st = SOLVERS[kind](s.apply, be, 1e-13)
    assert _ok(st)
    m, idx = s.dense()
    want = np.linalg.solve(m, be.reshape(3, -1)[:, idx].T).T
    assert np.abs(x.reshape(3, -1)[:, idx] - want).max() < 1e-11 * np.abs(want).max()
    assert not np.any(s.po(x))


@pytest.mark.parametrize("kind", list(SOLVERS))
def test_exact_inverse_preconditioner_converges_in_one_iteration(kind):
    dims, bc, kappa, eps = CASES[0]
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, eps, 1201))
    a_inv = np.linalg.inv(d.dense("D"))
    b = synth.gaussian_spinors(dims, bc, 2, 2201)
    k_inv = lambda v: (a_inv @ v.reshape(-1)).reshape(v.shape)
    x, st = SOLVERS[kind](d.D, b, 1e-12, precond=k_inv)
    its = [s.iters for s in st] if isinstance(st, list) else [st.iters]
    assert all(i == 1 for i in its), its
    assert _ok(st)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_block_and_global_forms_reduce_to_plain_bicgstab_for_one_rhs(k):
    """With one right-hand side the Frobenius products are ordinary inner
    products and the s x s systems are 1 x 1: all three forms produce the same
    iterate after k iterations."""
    dims, bc, kappa, eps = CASES[1]
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, eps, 1202))
    b = synth.gaussian_spinors(dims, bc, 1, 2202)
    xp, _ = bi.bicgstab(d.D, b, 1e-30, max_iter=k)
    xg, _ = bi.gl_bicgstab(d.D, b, 1e-30, max_iter=k)
    xb, _ = bi.bl_bicgstab(d.D, b, 1e-30, max_iter=k)
    scale = np.linalg.norm(xp)
    assert np.linalg.norm(xg - xp) < 1e-12 * scale
    assert np.linalg.norm(xb - xp) < 1e-12 * scale


def test_block_form_shares_the_krylov_space():
    """The block form converges in fewer iterations than the slowest RHS of
    the plain form on a rougher lattice (the effect the paper measures for
    Bl-BiCGStab); all solutions meet the tolerance."""
    dims, bc, kappa = (4, 4, 2, 4), "sf", 0.13
    d = WilsonDirac(dims, bc, kappa, synth.random_links(dims, bc, 0.5, 1203))
    s = schur.Schur(d)
    b = s.pe(synth.gaussian_spinors(dims, bc, 4, 2203))
    _, stp = bi.bicgstab(s.apply, b, 1e-10)
    _, stb = bi.bl_bicgstab(s.apply, b, 1e-10)
    assert _ok(stp) and _ok(stb)
    assert stb.iters < max(x.iters for x in stp)
