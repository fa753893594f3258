"""GPU parity of block CG (solver selection "blockcg") against the FP64 oracle.

Block CG reaches the same solutions as per-RHS CG, x_i = (D^+D)^-1 b_i, so
the oracle is that definition: every solution's FP64 residual is re-measured
with the oracle's operator and its error compared with the oracle's CG
solution within cond(D^+D) * (tol_gpu + tol_oracle) + 1e-14.  Sharing the
Krylov space must not cost iterations: block CG takes no more than the
slowest RHS of the batched CG on the same right-hand sides (up to rounding
for a single RHS, where the two are the same method).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import solvers
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


CASES = [
    ((4, 4, 4, 8), "sf", 0.13, 0.3, 1),
    ((4, 4, 4, 8), "sf", 0.13, 0.3, 3),
    ((4, 6, 2, 10), "sf", 0.13, 0.4, 5),
    ((6, 2, 4, 6), "periodic", 0.12, 0.5, 8),      # 72 sites per parity: ragged workgroup
    ((4, 4, 2, 6), "antiperiodic", 0.12, 0.5, 4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}_n{c[4]}")
def test_block_cg_matches_oracle(case):
    dims, bc, kappa, eps, n = case
    tol = 1e-10
    u = synth.random_links(dims, bc, eps, 1200 + n)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    d = WilsonDirac(dims, bc, kappa, u)
    b = synth.gaussian_spinors(dims, bc, n, 2200 + n)
    xb, sb, rcb = lat.solve(to_dev(b), tol=tol, prec="fp64", precond="blockcg", max_iter=5000)
    xc, sc, rcc = lat.solve(to_dev(b), tol=tol, prec="fp64", max_iter=5000)
    it_block = sb[0]["iters"]
    it_cg = max(s["iters"] for s in sc)
    res_str = ", ".join("%.2e" % s["true_rel_resid"] for s in sb)
    note(f"block CG n={n}: rc {rcb} iters {it_block} (batched CG max {it_cg}), true residuals {res_str}")
    assert rcb == 0 and all(s["status"] == 0 for s in sb), sb
    # with one RHS block CG is CG (its step lengths come from a 1x1 solve, so
    # rounding can move convergence by an iteration or two)
    assert it_block <= it_cg + (2 if n == 1 else 0), (it_block, it_cg)
    xb = to_host(xb)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(xb[i:i + 1])) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
        assert sb[i]["true_rel_resid"] <= tol
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = solvers.cg_cond(d.DdagD, b, 120)
    assert rel(xb, x_ref) <= c * (tol + 1e-14) + 1e-14, (rel(xb, x_ref), c)
    lat.close()


def test_block_cg_graph_replay_equals_eager_launches():
    """Two iterations are captured in a hipGraph and replayed between polls;
    launching the same kernels eagerly gives bitwise the same solution (odd
    max_iter covers the trailing single iteration)."""
    dims, bc, kappa, n = (4, 6, 2, 10), "sf", 0.13, 3
    u = synth.random_links(dims, bc, 0.4, 1300)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    b = to_dev(synth.gaussian_spinors(dims, bc, n, 2300))
    xg, sg, rcg = lat.solve(b, tol=1e-10, prec="fp64", precond="blockcg", max_iter=5000, use_graph=True)
    xe, se, rce = lat.solve(b, tol=1e-10, prec="fp64", precond="blockcg", max_iter=5000, use_graph=False)
    assert rcg == 0 and rce == 0
    assert sg[0]["iters"] == se[0]["iters"]
    assert np.array_equal(to_host(xg), to_host(xe))
    xo, so, rco = lat.solve(b, tol=1e-30, prec="fp64", precond="blockcg", max_iter=21, use_graph=True)
    assert rco == 1 and so[0]["iters"] == 21, so
    lat.close()


def test_block_cg_force_matches_batched_cg_force():
    """The force (Alg. 2) with block CG as its solver agrees with the force
    from batched CG: both solutions meet 1e-11, so the forces agree far
    inside 1e-8."""
    p = synth.CONFIG_1
    u = p.links()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    phi = to_dev(p.rhs())
    g_b, act_b, st_b, rc_b = lat.force(phi, tol=1e-11, prec="fp64", precond="blockcg", max_iter=5000)
    g_c, act_c, st_c, rc_c = lat.force(phi, tol=1e-11, prec="fp64", max_iter=5000)
    assert rc_b == 0 and rc_c == 0
    err = rel(to_host(g_b), to_host(g_c))
    note(f"force block vs batched CG: rel {err:.2e}; iters {st_b[0]['iters']} vs "
         f"{max(s['iters'] for s in st_c)}")
    assert err < 1e-8
    assert np.allclose(act_b, act_c, rtol=1e-9)
    lat.close()


def test_block_cg_rejects_bad_input():
    dims, bc = (4, 4, 4, 4), "sf"
    u = synth.random_links(dims, bc, 0.3, 1)
    lat = mfq.Lattice(dims, bc, 0.12, to_dev(u))
    b = to_dev(synth.gaussian_spinors(dims, bc, 2, 3))
    with pytest.raises(mfq.MfqError):
        lat.solve(b, prec="fp32", precond="blockcg")
    b9 = to_dev(synth.gaussian_spinors(dims, bc, 9, 4))
    with pytest.raises(mfq.MfqError):
        lat.solve(b9, prec="fp64", precond="blockcg")
    lat.close()
