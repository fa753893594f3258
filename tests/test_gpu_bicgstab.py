"""GPU parity of the paper's solver family (per-RHS, global and block
BiCGStab on the even/odd-preconditioned operator, in FP64 and with the FP32
inner solve as preconditioner) against the FP64 oracle: D x = b and
D^+ x = b with their residuals re-measured by the oracle and the error
bounded against the oracle's solution, the normal-equation solve built from
two of them, and the force of Alg. 2 through them."""
import sys

import numpy as np
import pytest

import synth
from oracle import force as fmod
from oracle import native, solvers
from oracle.dirac import WilsonDirac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1009_5169_amd as mfq  # noqa: E402

DEV = "cuda:0"
KINDS = ["bicgstab", "gl_bicgstab", "bl_bicgstab"]


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


CASES = [((4, 4, 4, 8), "sf", 0.13, 0.3, 3), ((6, 2, 4, 6), "periodic", 0.11, 0.5, 2),
         ((4, 6, 2, 4), "antiperiodic", 0.12, 0.5, 5)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}_n{c[4]}")
def test_solve_dirac_matches_oracle(case, kind, prec):
    dims, bc, kappa, eps, n = case
    u = synth.random_links(dims, bc, eps, 1300)
    d = WilsonDirac(dims, bc, kappa, u)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    b = synth.gaussian_spinors(dims, bc, n, 2300)
    c = np.sqrt(solvers.cg_cond(d.DdagD, b, 120))   # cond(D) ~ sqrt(cond(D^+D))
    tol = 1e-10
    for dagger, op, want_fn in ((False, d.D, solvers.solve_D), (True, d.Ddag, solvers.solve_Ddag)):
        x, st, rc = lat.solve_dirac(to_dev(b), dagger=dagger, precond=kind, prec=prec, tol=tol, max_iter=3000)
        assert rc == 0, st
        x = to_host(x)
        res = [rel(op(x[i:i + 1]), b[i:i + 1]) for i in range(n)]
        x_ref, _ = want_fn(d, b, 1e-14)
        err = rel(x, x_ref)
        note(f"{kind} {prec} {dims} {bc} dagger={dagger}: iters {st[0]['iters']} inner "
             f"{st[0]['inner_iters']}/{st[0]['inner_calls']} restarts {st[0]['reliable_updates']} "
             f"residuals {max(res):.2e} error {err:.2e}")
        assert max(res) <= 3 * tol, res
        assert err <= 3 * c * tol + 1e-14, (err, c)
        assert all(s["status"] == 0 and s["true_rel_resid"] <= tol for s in st)
        if prec == "fp32":
            assert st[0]["inner_calls"] >= 2 and st[0]["inner_iters"] > 0
        else:
            assert st[0]["inner_calls"] == 0
    lat.close()


@pytest.mark.parametrize("kind", KINDS)
def test_normal_solve_through_bicgstab(kind):
    dims, bc, kappa, eps, n = CASES[0]
    u = synth.random_links(dims, bc, eps, 1310)
    d = WilsonDirac(dims, bc, kappa, u)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    b = synth.gaussian_spinors(dims, bc, n, 2310)
    x, st, rc = lat.solve(to_dev(b), precond=kind, prec="fp64", tol=1e-12, max_iter=3000)
    assert rc == 0, st
    x = to_host(x)
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = solvers.cg_cond(d.DdagD, b, 120)
    for i in range(n):
        r = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert abs(st[i]["true_rel_resid"] - r) <= 0.01 * r + 1e-16
        assert r <= 10 * c * 1e-12
    assert rel(x, x_ref) <= 100 * c * 1e-12
    lat.close()


@pytest.mark.parametrize("kind,prec", [("gl_bicgstab", "fp32"), ("bl_bicgstab", "fp64"), ("bicgstab", "fp64")])
def test_force_through_bicgstab_matches_oracle(kind, prec):
    """Alg. 2 with the paper's solvers (D X = Phi, D^+ Y = X) on the 8^3x8 SF
    5-RHS case, solves to 1e-12: X, Y, the force and the action against the
    oracle's Alg. 2 (forces within 1e-8, solutions within 1e-9)."""
    p = synth.CONFIG_1
    u, phi = p.links(), p.rhs()
    nd = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    x_ref, _ = solvers.solve_D(nd, phi, 1e-13)
    y_ref, _ = solvers.solve_Ddag(nd, x_ref, 1e-13)
    g_ref = fmod.coefficients_to_matrix(fmod.force_coefficients(WilsonDirac(p.dims, p.bc, p.kappa, u), x_ref, y_ref))
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    g, a, stats, rc, x, y = lat.force(to_dev(phi), tol=1e-12, prec=prec, precond=kind, want_xy=True, max_iter=5000)
    assert rc == 0, stats
    eg, ex, ey = rel(to_host(g), g_ref), rel(to_host(x), x_ref), rel(to_host(y), y_ref)
    note(f"force via {kind} {prec}: G {eg:.2e} X {ex:.2e} Y {ey:.2e}; iters {stats[0]['iters']} "
         f"inner {stats[0]['inner_iters']}/{stats[0]['inner_calls']}")
    assert eg < 1e-8 and ex < 1e-9 and ey < 1e-9
    np.testing.assert_allclose(a, fmod.action(None, x_ref), rtol=1e-9)
    lat.close()


def test_bicgstab_rejects_fp16_and_too_many_rhs():
    dims, bc = (4, 4, 4, 4), "sf"
    u = synth.random_links(dims, bc, 0.3, 1320)
    lat = mfq.Lattice(dims, bc, 0.125, to_dev(u))
    b = to_dev(synth.gaussian_spinors(dims, bc, 9, 2320))
    with pytest.raises(mfq.MfqError):
        lat.solve_dirac(b[:2].contiguous(), precond="bl_bicgstab", prec="fp16")
    with pytest.raises(mfq.MfqError):
        lat.solve_dirac(b, precond="gl_bicgstab", prec="fp64")
    with pytest.raises(mfq.MfqError):
        lat.solve_dirac(b[:2].contiguous(), precond="blockcg", prec="fp64")
    lat.close()
