"""GPU parity at the full size of the comparison rows (16^3x16 SF, 5 RHS), in
the launch configurations the benchmark times (the shipped tuning table).

At this size the oracle is the compiled FP64 reference operator (oracle/native)
and the numpy network: every solution's residual is re-measured with the
oracle's D^+D, the FP64 operator is compared element by element, and the
network application is compared with the oracle's forward pass.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import native, ptc
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


def test_full_size_solves_and_operator():
    p = synth.CONFIG_2
    u = p.links()
    b = p.rhs()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    got = to_host(lat.dslash("D", to_dev(b)))
    err = rel(got, d.D(b))
    note(f"{p.name}: FP64 D rel err {err:.2e}")
    assert err < 1e-13
    for prec, pc in (("fp64", "none"), ("fp32", "none"), ("fp16", "none"), ("fp64", "blockcg")):
        x, st, rc = lat.solve(to_dev(b), tol=1e-10, prec=prec, precond=pc, max_iter=20000)
        assert rc == 0, (prec, pc, st)
        x = to_host(x)
        r = b - d.DdagD(x)
        res = [float(np.linalg.norm(r[i]) / np.linalg.norm(b[i])) for i in range(p.n_rhs)]
        note(f"{p.name} {prec} {pc}: iters {[s['iters'] for s in st]} oracle residuals "
             + ", ".join("%.2e" % v for v in res))
        assert max(res) <= 1.05e-10
    lat.close()


def test_full_size_network_application():
    """The matrix-core network on a 16^3x16 field against the oracle's
    forward pass with the same BF16-valued weights."""
    p = synth.CONFIG_4
    u = p.links()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    lat.precond_init(seed=5)
    w = lat.precond_get_weights("inference")
    w1 = w[: 9 * 8 * 16].reshape(9, 8, 4, 4)[:, :, None]
    w2 = w[9 * 8 * 16:].reshape(9, 8, 4, 4)[:, None]
    r = synth.gaussian_spinors(p.dims, p.bc, 1, 2500)
    got = to_host(lat.precond_apply(to_dev(r)))
    want, _ = ptc.forward(ptc.Transport(WilsonDirac(p.dims, p.bc, p.kappa, u)), w1, w2, r)
    err = rel(got, want)
    note(f"{p.name}: network application rel err {err:.2e}")
    assert err < 2e-5
    lat.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
def test_bandwidth_lattice_operator(prec, tol):
    """D on the 32^3x64 periodic lattice of the benchmark's bandwidth runs, one
    RHS, in the launch shape the benchmark times (the tuned shape of the
    solver's hopping kernel), against the compiled oracle over every site."""
    import bench
    dims = (32, 32, 32, 64)
    u = bench.bandwidth_links(dims, synth, np)
    lat = mfq.Lattice(dims, "periodic", bench.BANDWIDTH_KAPPA, to_dev(u))
    x = synth.gaussian_spinors(dims, "periodic", 1, 2600)
    got = to_host(lat.dslash("D", to_dev(x), prec=prec))
    want = native.NativeWilson(dims, "periodic", bench.BANDWIDTH_KAPPA, u).D(x)
    err = rel(got, want)
    note(f"32^3x64 {prec} D (shape {lat.hop_shape(prec, 1)}): rel err {err:.2e}")
    assert err < tol
    lat.close()


# every bandwidth run the benchmark reports besides the 1-RHS FP64 / FP32 cases
# above: lattice, boundary, precision, RHS, tolerance of the relative error
# (FP16 storage rounds the input and the output to 11 significant bits: 2 x 2^-11)
BANDWIDTH_RUNS = [
    ((32, 32, 32, 64), "periodic", "fp64", 5, 1e-13),
    ((32, 32, 32, 64), "periodic", "fp64", 8, 1e-13),
    ((32, 32, 32, 64), "periodic", "fp32", 5, 2e-6),
    ((32, 32, 32, 64), "periodic", "fp32", 8, 2e-6),
    ((32, 32, 32, 64), "periodic", "fp16", 1, 1e-3),
    ((32, 32, 32, 64), "periodic", "fp16", 5, 1e-3),
    ((32, 32, 32, 64), "periodic", "fp16", 8, 1e-3),
    ((48, 48, 48, 48), "periodic", "fp32", 1, 2e-6),
    ((48, 48, 48, 48), "periodic", "fp32", 5, 2e-6),
    ((32, 32, 32, 64), "sf", "fp32", 5, 2e-6),
]


@pytest.mark.parametrize("dims,bc,prec,n_rhs,tol", BANDWIDTH_RUNS,
                         ids=[f"{'x'.join(map(str, c[0]))}-{c[1]}-{c[2]}-{c[3]}rhs" for c in BANDWIDTH_RUNS])
def test_bandwidth_lattice_operator_as_timed(dims, bc, prec, n_rhs, tol):
    """D on the benchmark's bandwidth lattices in the launch shape it times
    (the tuned shape for that precision and RHS count, e.g. the 5-RHS FP32
    shape of the HBM-resident roofline entry), against the compiled oracle
    over every site and RHS."""
    import bench
    u = bench.bandwidth_links(dims, synth, np, bc)
    lat = mfq.Lattice(dims, bc, bench.BANDWIDTH_KAPPA, to_dev(u))
    x = synth.gaussian_spinors(dims, bc, n_rhs, 2610)
    got = to_host(lat.dslash("D", to_dev(x), prec=prec))
    want = native.NativeWilson(dims, bc, bench.BANDWIDTH_KAPPA, u).D(x)
    shape = lat.hop_shape(prec, n_rhs)
    for i in range(n_rhs):
        err = rel(got[i], want[i])
        note(f"{dims} {bc} {prec} D rhs {i} (shape {shape}): rel err {err:.2e}")
        assert err < tol
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_learned_solve_matches_oracle(prec):
    """The learned row at full size (16^3x16 SF, kappa 0.1375, 5 RHS): a
    network trained briefly on the GPU, FGMRES(16) with it (the cycle in FP64
    or in FP32 with FP64 restarts) to the parity
    tolerance min(1e-10, 3e-10 / cond) (cond from the oracle's Lanczos
    estimate), every residual re-measured with the oracle's operator, and the
    first RHS's solution within 1e-9 of the oracle's own CG solution."""
    from oracle import solvers
    p = synth.CONFIG_4
    u, b = p.links(), p.rhs()
    d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    xi = to_dev(synth.gaussian_spinors(p.dims, p.bc, 4, synth.PTC_TRAIN_SEED))
    r, e = lat.precond_pairs(xi, every=5, n_snap=4)
    lat.precond_init(seed=1)
    hist = lat.precond_train(r, e, steps=100, lr=3e-3)
    cond = solvers.cg_cond(d.DdagD, b[:1], 150)
    tol = min(1e-10, 3e-10 / cond)  # the Lanczos estimate bounds cond from below
    note(f"{p.name}: training loss {hist[0]:.3f} -> {hist[-1]:.3f}; cond ~ {cond:.0f}, parity tol {tol:.2e}")
    x, st, rc = lat.solve(to_dev(b), tol=tol, prec=prec, precond="ptc", max_iter=50000)
    assert rc == 0, st
    x = to_host(x)
    res = [float(np.linalg.norm((b[i:i + 1] - d.DdagD(x[i:i + 1]))) / np.linalg.norm(b[i]))
           for i in range(p.n_rhs)]
    note(f"{p.name} fgmres+ptc {prec}: iters {[s['iters'] for s in st]} oracle residuals "
         + ", ".join("%.2e" % v for v in res))
    assert max(res) <= 1.05 * tol
    x_ref, _ = solvers.cg(d.DdagD, b[:1], 1e-13)
    err = rel(x[:1], x_ref)
    note(f"{p.name} fgmres+ptc {prec}: RHS 0 error against the oracle's CG solution {err:.2e}")
    assert err < 1e-9
    lat.close()
