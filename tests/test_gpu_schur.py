"""GPU parity of the even/odd Schur-complement path against the FP64 oracle:
the operators D^, D^^+ and D^^+D^ element by element in every precision, CG
solves through the Schur complement (route S) with their residual re-measured
by the oracle and a cond-bounded error against the oracle's solution, the
force of Alg. 2 through route S, and the even/odd action variant's force and
action."""
import sys

import numpy as np
import pytest

import synth
from oracle import force as fmod
from oracle import native, schur, solvers
from oracle.dirac import WilsonDirac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1009_5169_amd as mfq  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make(dims, bc, kappa, eps, seed):
    u = synth.random_links(dims, bc, eps, seed)
    return u, mfq.Lattice(dims, bc, kappa, to_dev(u)), WilsonDirac(dims, bc, kappa, u)


LATTICES = [
    ((4, 4, 4, 4), "sf", 0.125, 0.3),
    ((8, 8, 8, 8), "sf", 0.13, 0.3),
    ((6, 2, 4, 6), "periodic", 0.12, 0.5),    # 72 sites per parity: ragged tiles
    ((4, 6, 2, 4), "antiperiodic", 0.12, 0.5),
]


@pytest.mark.parametrize("case", LATTICES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}")
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6), ("fp16", 1e-2)])
def test_schur_operators(case, prec, tol):
    dims, bc, kappa, eps = case
    note(f"schur operators {prec} {dims} {bc}")
    _, lat, d = make(dims, bc, kappa, eps, 1000)
    s = schur.Schur(d)
    psi = synth.gaussian_spinors(dims, bc, 3, 2300)
    x = to_dev(psi)
    want = {"schur": s.apply(psi), "schur_dag": s.apply(psi, dagger=True), "schur_normal": s.normal(psi)}
    for op, w in want.items():
        got = to_host(lat.dslash(op, x, prec=prec))
        assert rel(got, w) < tol, (op, rel(got, w))
        assert not np.any(s.po(got)), op      # the odd sites are zero
    lat.close()


def _cond(d, b):
    return solvers.cg_cond(d.DdagD, b, 120)


SOLVE_CASES = [
    (synth.CONFIG_0.dims, "sf", 0.125, 0.3, 1),
    ((4, 4, 4, 8), "sf", 0.13, 0.3, 3),
    ((6, 2, 4, 6), "periodic", 0.11, 0.5, 2),
    ((4, 6, 2, 4), "antiperiodic", 0.12, 0.5, 2),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("case", SOLVE_CASES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}_n{c[4]}")
def test_route_s_solve_matches_oracle(case, prec):
    """x = (D^+D)^-1 b by two Schur solves, each to 1e-12 on its own normal
    equations: the full system's FP64 residual the library reports equals the
    oracle's measurement, and residual and solution error stay within
    cond(D^+D) times 10 and 100 times that tolerance (each Schur solve's error
    is bounded by the condition number of its normal operator, and the
    second solve carries the first one's error through D^-1)."""
    dims, bc, kappa, eps, n = case
    tol = 1e-12
    note(f"route S solve {prec} {dims} {bc} n={n}")
    _, lat, d = make(dims, bc, kappa, eps, 1010)
    b = synth.gaussian_spinors(dims, bc, n, 2010)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec=prec, route="schur", max_iter=5000)
    assert rc == 0, stats
    x = to_host(x)
    c = _cond(d, b)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert abs(stats[i]["true_rel_resid"] - res) <= 0.01 * res + 1e-16, (stats[i], res)
        assert res <= 10 * c * tol, (i, res, c)
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    assert rel(x, x_ref) <= 100 * c * tol, (rel(x, x_ref), c)
    note(f"  iters {[s['iters'] for s in stats]}, full residuals "
         f"{[round(s['true_rel_resid'], 14) for s in stats]}, error {rel(x, x_ref):.2e} (cond {c:.0f})")
    lat.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-13), ("fp16", 1e-11)])
def test_route_s_force_matches_oracle(prec, tol):
    """Alg. 2 through the Schur complement (D X = Phi, D^+ Y = X) on the
    8^3x8 SF 5-RHS case, solves to 1e-13 (FP16 storage: 1e-11): X, Y, the
    force and the action against the oracle's Alg. 2 (forces within 1e-8,
    solutions within 1e-9)."""
    p = synth.CONFIG_1
    u, phi = p.links(), p.rhs()
    nd = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    x_ref, _ = solvers.solve_D(nd, phi, 1e-13)
    y_ref, _ = solvers.solve_Ddag(nd, x_ref, 1e-13)
    g_ref = fmod.coefficients_to_matrix(fmod.force_coefficients(WilsonDirac(p.dims, p.bc, p.kappa, u), x_ref, y_ref))
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    g, a, stats, rc, x, y = lat.force(to_dev(phi), tol=tol, prec=prec, route="schur", want_xy=True)
    assert rc == 0, stats
    eg, ex, ey = rel(to_host(g), g_ref), rel(to_host(x), x_ref), rel(to_host(y), y_ref)
    note(f"route S force {prec}: G {eg:.2e} X {ex:.2e} Y {ey:.2e}, iters {[s['iters'] for s in stats]}")
    assert eg < 1e-8 and ex < 1e-9 and ey < 1e-9
    np.testing.assert_allclose(a, fmod.action(None, x_ref), rtol=1e-9)
    lat.close()


@pytest.mark.parametrize("case", [((4, 4, 4, 4), "sf", 0.125, 0.3, 2, "fp64"),
                                  ((4, 4, 4, 8), "sf", 0.13, 0.3, 3, "fp32"),
                                  ((4, 2, 2, 4), "antiperiodic", 0.12, 0.5, 2, "fp64")],
                         ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}_{c[5]}")
def test_eo_action_force_matches_oracle(case):
    """The even/odd action variant: force, full-lattice X and Y and the action
    |X_e|^2 against the oracle's eo_force (CG to 1e-14)."""
    dims, bc, kappa, eps, n, prec = case
    u, lat, d = make(dims, bc, kappa, eps, 1020)
    phi = synth.gaussian_spinors(dims, bc, n, 2020)
    g, a, stats, rc, x, y = lat.force(to_dev(phi), tol=1e-12, prec=prec, eo_action=True, want_xy=True)
    assert rc == 0, stats
    g_ref, a_ref, x_ref, y_ref = schur.eo_force(d, phi, tol=1e-14)
    eg, ex, ey = rel(to_host(g), g_ref), rel(to_host(x), x_ref), rel(to_host(y), y_ref)
    note(f"eo action {prec} {dims}: G {eg:.2e} X {ex:.2e} Y {ey:.2e}, iters {[s['iters'] for s in stats]}")
    bound = 1e-9 if prec == "fp64" else 1e-8
    assert eg < bound and ex < bound and ey < bound
    np.testing.assert_allclose(a, a_ref, rtol=bound)
    # the force kernel fed the same X, Y: FP64 parity at 1e-12
    g_same = fmod.coefficients_to_matrix(fmod.force_coefficients(d, to_host(x), to_host(y)))
    assert rel(to_host(g), g_same) < 1e-12
    lat.close()


def test_route_s_rejects_other_solvers():
    dims, bc = (4, 4, 4, 4), "sf"
    _, lat, _ = make(dims, bc, 0.125, 0.3, 1030)
    b = to_dev(synth.gaussian_spinors(dims, bc, 1, 2030))
    with pytest.raises(mfq.MfqError) as e:
        lat.solve(b, route="schur", precond="blockcg", prec="fp64")
    assert e.value.code == -1
    lat.close()
