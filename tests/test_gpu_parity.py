"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (relative, global 2-norm over the whole field and all RHS):
* single FP64 operator applications and the force kernel fed with the same
  X, Y: 1e-12;
* FP32 operators: 2e-6 (a few units of FP32 rounding over the 8-term stencil);
* FP16-storage operators: 1e-2 (FP16 rounding of spinors and links);
* solves: the solution error is bounded by cond(D^+D) times the residual, so a
  solve is compared with |x - x_oracle| / |x_oracle| <= cond * (tol_gpu +
  tol_oracle) + 1e-14, and its FP64 residual is re-measured with the oracle.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import force as fmod
from oracle import solvers
from oracle.dirac import GAMMA5, WilsonDirac, even_odd_mask

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
    ((4, 4, 4, 4), "sf", 0.125, 0.3),       # the 4^4 SF case
    ((8, 8, 8, 8), "sf", 0.13, 0.3),        # the 8^3x8 SF case
    ((6, 2, 4, 6), "periodic", 0.12, 0.5),  # ragged: 72 sites per parity
    ((4, 6, 2, 4), "antiperiodic", 0.12, 0.5),
    ((2, 2, 6, 6), "sf", 0.13, 0.5),
]


@pytest.mark.parametrize("case", LATTICES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}")
@pytest.mark.parametrize("n_rhs", [1, 5, 9])
def test_operators_fp64(case, n_rhs):
    dims, bc, kappa, eps = case
    note(f"operators fp64 {dims} {bc} n_rhs={n_rhs}")
    _, lat, d = make(dims, bc, kappa, eps, 1000)
    psi = synth.gaussian_spinors(dims, bc, n_rhs, 2000 + n_rhs)
    x = to_dev(psi)
    even = even_odd_mask(dims, bc)[None, ..., None, None]
    want = {
        "D": d.D(psi), "Ddag": d.Ddag(psi), "DdagD": d.DdagD(psi),
        "hop": d.hop(psi), "hop_dag": d.hop(psi, dagger=True),
        "hop_eo": np.where(even, d.hop(np.where(even, 0, psi)), 0),
        "hop_oe": np.where(even, 0, d.hop(np.where(even, psi, 0))),
    }
    for op, w in want.items():
        got = to_host(lat.dslash(op, x))
        assert rel(got, w) < 1e-13, op
    lat.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("fp16", 1e-2)])
def test_operators_reduced_precision(prec, tol):
    for dims, bc, kappa, eps in LATTICES[:3]:
        note(f"operators {prec} {dims} {bc}")
        _, lat, d = make(dims, bc, kappa, eps, 1000)
        psi = synth.gaussian_spinors(dims, bc, 5, 2100)
        x = to_dev(psi)
        even = even_odd_mask(dims, bc)[None, ..., None, None]
        want = {"D": d.D, "Ddag": d.Ddag, "hop": d.hop, "DdagD": d.DdagD,
                "hop_dag": lambda f: d.hop(f, dagger=True),
                "hop_eo": lambda f: np.where(even, d.hop(np.where(even, 0, f)), 0),
                "hop_oe": lambda f: np.where(even, 0, d.hop(np.where(even, f, 0)))}
        for op, w in want.items():
            got = to_host(lat.dslash(op, x, prec=prec))
            ref = w(psi)
            assert rel(got, ref) < tol, (op, rel(got, ref))
        lat.close()


def test_fp16_scale_extremes():
    """The per-site norm keeps FP16 storage finite for inputs of 1e+-30."""
    dims, bc = (4, 4, 4, 4), "sf"
    _, lat, d = make(dims, bc, 0.125, 0.3, 1000)
    psi = synth.gaussian_spinors(dims, bc, 2, 7)
    psi[0] *= 1e30
    psi[1] *= 1e-30
    got = to_host(lat.dslash("D", to_dev(psi), prec="fp16"))
    assert np.all(np.isfinite(got))
    for i in range(2):
        assert rel(got[i], d.D(psi[i:i + 1])[0]) < 1e-2
    lat.close()


def _cond(d, b):
    return solvers.cg_cond(d.DdagD, b, 120)


SOLVE_CASES = [
    (synth.CONFIG_0.dims, "sf", 0.125, 0.3, 1, 1e-12),
    ((4, 4, 4, 8), "sf", 0.13, 0.3, 3, 1e-10),
    ((6, 2, 4, 6), "periodic", 0.11, 0.5, 2, 1e-10),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("case", SOLVE_CASES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}_n{c[4]}")
def test_solve_matches_oracle(case, prec):
    dims, bc, kappa, eps, n, tol = case
    note(f"solve {prec} {dims} {bc} n={n} tol={tol}")
    _, lat, d = make(dims, bc, kappa, eps, 1000)
    b = synth.gaussian_spinors(dims, bc, n, 2000)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec=prec, max_iter=5000)
    assert rc == 0, stats
    x = to_host(x)
    # FP64 residual of the GPU solution, measured by the oracle
    for i in range(n):
        r = b[i:i + 1] - d.DdagD(x[i:i + 1])
        res = np.linalg.norm(r) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
        assert stats[i]["true_rel_resid"] <= tol and stats[i]["status"] == 0
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = _cond(d, b)
    assert rel(x, x_ref) <= c * (tol + 1e-14) + 1e-14, (rel(x, x_ref), c)
    lat.close()


BC_CODE = {"sf": 0, "periodic": 1, "antiperiodic": 2}
PREC_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(64, 1, 0, 2, 0), (64, 3, 1, 4, 0), (128, 2, 0, 8, 0), (64, 1, 1, 16, 0),
                                   (128, 1, 0, 0, 0), (64, 3, 1, 0, 0), (64, 1, 0, 0, 2), (64, 1, 1, 0, 4),
                                   (64, 3, 0, 0, 2), (64, 2, 1, 0, 2), (64, 3, 4, 0, 0), (128, 2, 5, 0, 0)],
                         ids=lambda s: "sb%d_nr%d_xcd%d_tc%d_ds%d" % s)
def test_forced_launch_shapes_match_oracle(tmp_path, monkeypatch, shape, prec):
    """Every launch shape the autotuner may pick, forced through the tuning
    cache: plain, time-sweep (sweep lengths that do not divide the 9 dynamical
    time slices) and direction-split both-parity kernels, with and without the
    XCD remap, give solutions that meet the oracle's residual and error bound."""
    dims, bc, kappa, n, tol = (4, 6, 2, 10), "sf", 0.13, 3, 1e-10
    key = "gfx950 %d %d %d %d %d %d %d" % (dims + (BC_CODE[bc], n, PREC_BYTES[prec]))
    cache = tmp_path / "tune.txt"
    cache.write_text(key + "|%d %d %d %d %d\n" % shape)
    monkeypatch.setenv("MFQ_AUTOTUNE_CACHE", str(cache))
    _, lat, d = make(dims, bc, kappa, 0.4, 1100)
    b = synth.gaussian_spinors(dims, bc, n, 2100)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec=prec, max_iter=5000)
    assert tuple(lat.hop_shape(prec, n)) == shape
    assert rc == 0, stats
    x = to_host(x)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = _cond(d, b)
    assert rel(x, x_ref) <= c * (tol + 1e-14) + 1e-14, (rel(x, x_ref), c)
    lat.close()


def test_fp32_split_shape_too_wide_for_fp64(tmp_path, monkeypatch):
    """A direction-split FP32 shape (4 wavefronts x 2 RHS rows) whose LDS
    partial sums fit at FP32 width but not at FP64 width: the FP64
    true-residual launches of the reliable updates must not use it as is.
    Solutions meet the oracle's residual and error bound."""
    dims, bc, kappa, n, tol = (4, 6, 2, 10), "sf", 0.13, 3, 1e-10
    shape = (64, 2, 0, 0, 4)
    key = "gfx950 %d %d %d %d %d %d %d" % (dims + (BC_CODE[bc], n, PREC_BYTES["fp32"]))
    cache = tmp_path / "tune.txt"
    cache.write_text(key + "|%d %d %d %d %d\n" % shape)
    monkeypatch.setenv("MFQ_AUTOTUNE_CACHE", str(cache))
    _, lat, d = make(dims, bc, kappa, 0.4, 1120)
    b = synth.gaussian_spinors(dims, bc, n, 2120)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec="fp32", max_iter=5000)
    assert tuple(lat.hop_shape("fp32", n)) == shape
    assert rc == 0, stats
    assert all(s["reliable_updates"] >= 2 for s in stats)
    x = to_host(x)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = _cond(d, b)
    assert rel(x, x_ref) <= c * (tol + 1e-14) + 1e-14, (rel(x, x_ref), c)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(64, 1, 2, 0, 0), (64, 3, 3, 0, 0), (64, 1, 2, 0, 4), (64, 2, 3, 0, 2),
                                   (128, 1, 3, 0, 0), (64, 3, 7, 0, 0)],
                         ids=lambda s: "sb%d_nr%d_xcd%d_tc%d_ds%d" % s)
@pytest.mark.parametrize("lattice", [((8, 16, 6, 6), "sf"), ((8, 16, 4, 4), "periodic")],
                         ids=["sf8x16x6x6", "periodic8x16x4x4"])
def test_z_blocked_tile_order_matches_oracle(tmp_path, monkeypatch, lattice, shape, prec):
    """The z-blocked tile order (bit 1 of the order flags) on lattices whose
    (z, t) planes hold whole 64-site tiles: blocks of 2 z values over 5 SF
    time slices and of 4 over 4 periodic ones, with and without the XCD
    remap, plain and direction-split kernels; 128-site tiles do not divide the
    64-site planes, so that shape keeps the half-index order.  Solutions meet
    the oracle's residual and error bound."""
    dims, bc = lattice
    kappa, n, tol = 0.13, 3, 1e-10
    key = "gfx950 %d %d %d %d %d %d %d" % (dims + (BC_CODE[bc], n, PREC_BYTES[prec]))
    cache = tmp_path / "tune.txt"
    cache.write_text(key + "|%d %d %d %d %d\n" % shape)
    monkeypatch.setenv("MFQ_AUTOTUNE_CACHE", str(cache))
    _, lat, d = make(dims, bc, kappa, 0.4, 1110)
    b = synth.gaussian_spinors(dims, bc, n, 2110)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec=prec, max_iter=5000)
    assert tuple(lat.hop_shape(prec, n)) == shape
    assert rc == 0, stats
    x = to_host(x)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = _cond(d, b)
    assert rel(x, x_ref) <= c * (tol + 1e-14) + 1e-14, (rel(x, x_ref), c)
    lat.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("shape,lattice", [
    ((64, 3, 8, 0, 0), ((4, 6, 2, 10), "sf")), ((128, 2, 9, 0, 0), ((4, 6, 2, 10), "sf")),
    ((256, 3, 8, 0, 0), ((6, 2, 4, 6), "periodic")), ((64, 2, 11, 0, 0), ((8, 16, 6, 6), "sf")),
    ((64, 3, 10, 0, 0), ((8, 16, 4, 4), "periodic"))],
    ids=lambda v: "sb%d_nr%d_xcd%d_tc%d_ds%d" % v if len(v) == 5 else f"{v[1]}{'x'.join(map(str, v[0]))}")
def test_rhs_in_thread_shapes_match_oracle(tmp_path, monkeypatch, shape, lattice, prec):
    """The RHS-in-thread hopping kernel (order flag bit 3: each thread one site
    for nr RHS, links loaded once per thread), forced through the tuning cache:
    groups of 2 over 3 RHS (a ragged last group), workgroups of 64..256 sites,
    with the XCD remap and the z-blocked order.  Solutions meet the oracle's
    residual and error bound."""
    dims, bc = lattice
    kappa, n, tol = 0.13, 3, 1e-10
    key = "gfx950 %d %d %d %d %d %d %d" % (dims + (BC_CODE[bc], n, PREC_BYTES[prec]))
    cache = tmp_path / "tune.txt"
    cache.write_text(key + "|%d %d %d %d %d\n" % shape)
    monkeypatch.setenv("MFQ_AUTOTUNE_CACHE", str(cache))
    _, lat, d = make(dims, bc, kappa, 0.4, 1150)
    b = synth.gaussian_spinors(dims, bc, n, 2150)
    # the operator in the forced shape (both-parity launches), element by element
    for op in ("D", "Ddag"):
        got = to_host(lat.dslash(op, to_dev(b), prec=prec))
        want = d.D(b) if op == "D" else d.Ddag(b)
        assert rel(got, want) < (2e-6 if prec == "fp32" else 1e-2), (op, rel(got, want))
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec=prec, max_iter=5000)
    assert tuple(lat.hop_shape(prec, n)) == shape
    assert rc == 0, stats
    x = to_host(x)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
    x_ref, _ = solvers.cg_normal(d, b, 1e-14)
    c = _cond(d, b)
    assert rel(x, x_ref) <= c * (tol + 1e-14) + 1e-14, (rel(x, x_ref), c)
    lat.close()


@pytest.mark.parametrize("shape", [(64, 3, 4, 0, 0), (256, 2, 6, 0, 0)],
                         ids=lambda s: "sb%d_nr%d_xcd%d_tc%d_ds%d" % s)
def test_lds_link_tile_fp16_matches_oracle(tmp_path, monkeypatch, shape):
    """The LDS link tile (order flag bit 2) with FP16 storage: the FP16 links
    staged in LDS (4-half chunks), FP64 defect correction to 1e-10."""
    dims, bc, kappa, n, tol = (4, 6, 2, 10), "sf", 0.13, 3, 1e-10
    key = "gfx950 %d %d %d %d %d %d %d" % (dims + (BC_CODE[bc], n, PREC_BYTES["fp16"]))
    cache = tmp_path / "tune.txt"
    cache.write_text(key + "|%d %d %d %d %d\n" % shape)
    monkeypatch.setenv("MFQ_AUTOTUNE_CACHE", str(cache))
    _, lat, d = make(dims, bc, kappa, 0.4, 1140)
    b = synth.gaussian_spinors(dims, bc, n, 2140)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec="fp16", max_iter=5000)
    assert tuple(lat.hop_shape("fp16", n)) == shape
    assert rc == 0, stats
    x = to_host(x)
    for i in range(n):
        res = np.linalg.norm(b[i:i + 1] - d.DdagD(x[i:i + 1])) / np.linalg.norm(b[i])
        assert res <= tol * 1.05, (i, res)
    lat.close()


def test_solve_fp64_tight_matches_oracle_to_1e12():
    """On the 4^4 SF case (cond ~ 180) an FP64 solve to 1e-12/cond reproduces
    the oracle's solution to 1e-12."""
    p = synth.CONFIG_0
    u = p.links()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    d = WilsonDirac(p.dims, p.bc, p.kappa, u)
    b = p.rhs()
    c = _cond(d, b)
    tol = max(1e-12 / c, 2e-15)
    x, stats, rc = lat.solve(to_dev(b), tol=tol, prec="fp64", max_iter=5000)
    x_ref = solvers.dense_solve(d, b, "DdagD")
    note(f"tight fp64 solve: cond={c:.1f} tol={tol:.2e} err={rel(to_host(x), x_ref):.2e} rc={rc}")
    assert rel(to_host(x), x_ref) < 1e-12
    lat.close()


def test_solve_config1_residual_and_bound():
    """The 8^3x8 SF, 5-RHS case at 1e-10 in FP64, FP32+reliable and FP16: the
    oracle-measured residual of every RHS meets the tolerance."""
    p = synth.CONFIG_1
    u = p.links()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u))
    d = WilsonDirac(p.dims, p.bc, p.kappa, u)
    b = p.rhs()
    for prec in ("fp64", "fp32", "fp16"):
        x, stats, rc = lat.solve(to_dev(b), tol=1e-10, prec=prec, max_iter=10000)
        note(f"config1 {prec}: rc={rc} iters={[s['iters'] for s in stats]} "
             f"updates={[s['reliable_updates'] for s in stats]}")
        assert rc == 0
        x = to_host(x)
        r = b - d.DdagD(x)
        for i in range(p.n_rhs):
            assert np.linalg.norm(r[i]) / np.linalg.norm(b[i]) <= 1.05e-10
    lat.close()


def test_fp64_solve_is_bitwise_reproducible():
    p = synth.CONFIG_1
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(p.links()))
    b = to_dev(p.rhs())
    x1, s1, _ = lat.solve(b, tol=1e-10, prec="fp64")
    x2, s2, _ = lat.solve(b, tol=1e-10, prec="fp64")
    assert torch.equal(x1, x2)
    assert [s["iters"] for s in s1] == [s["iters"] for s in s2]
    lat.close()


def test_batched_equals_single_rhs_solves():
    dims, bc, kappa = (4, 4, 4, 8), "sf", 0.13
    _, lat, d = make(dims, bc, kappa, 0.3, 1000)
    b = synth.gaussian_spinors(dims, bc, 4, 2000)
    xb, _, _ = lat.solve(to_dev(b), tol=1e-12, prec="fp64")
    xb = to_host(xb)
    c = _cond(d, b)
    for i in range(4):
        xi, _, _ = lat.solve(to_dev(b[i:i + 1]), tol=1e-12, prec="fp64")
        assert rel(to_host(xi)[0], xb[i]) <= 2 * c * 1e-12
    lat.close()


def test_zero_rhs_and_not_converged():
    dims, bc, kappa = (4, 4, 4, 4), "sf", 0.125
    _, lat, _ = make(dims, bc, kappa, 0.3, 1000)
    b = synth.gaussian_spinors(dims, bc, 2, 5)
    b[1] = 0
    x, stats, rc = lat.solve(to_dev(b), tol=1e-12, prec="fp64", max_iter=5)
    assert rc == 1
    assert stats[0]["status"] == 1 and stats[0]["iters"] >= 5
    assert stats[1]["status"] == 0 and stats[1]["iters"] == 0
    assert not np.any(to_host(x)[1])
    lat.close()


def test_invalid_inputs_raise():
    dims, bc = (4, 4, 4, 4), "sf"
    u = synth.random_links(dims, bc, 0.3, 1)
    lat = mfq.Lattice(dims, bc, 0.125, to_dev(u))
    b = synth.gaussian_spinors(dims, bc, 1, 5)
    b[0, 1, 2, 3, 0, 1, 2] = np.nan
    with pytest.raises(mfq.MfqError) as e:
        lat.solve(to_dev(b), tol=1e-10)
    assert e.value.code == -1
    with pytest.raises(mfq.MfqError):
        lat.solve(to_dev(synth.gaussian_spinors(dims, bc, 1, 5)), tol=0.0)
    bad = u.copy()
    bad[0, 1, 0, 0, 0, 0, 0] = np.inf
    with pytest.raises(mfq.MfqError):
        mfq.Lattice(dims, bc, 0.125, to_dev(bad))
    with pytest.raises(mfq.MfqError):
        mfq.Lattice(dims, bc, 0.3, to_dev(u))
    # no right-hand sides: the library refuses n_rhs = 0 with an error
    empty = to_dev(synth.gaussian_spinors(dims, bc, 1, 5)[:0])
    for call in (lambda: lat.solve(empty, tol=1e-10), lambda: lat.dslash("D", empty)):
        with pytest.raises(mfq.MfqError) as e:
            call()
        assert e.value.code == -1
    lat.close()


@pytest.mark.parametrize("case", [(synth.CONFIG_0.dims, "sf", 0.125, 0.3, 1),
                                  ((4, 4, 4, 8), "sf", 0.13, 0.3, 3),
                                  ((4, 2, 2, 4), "antiperiodic", 0.12, 0.5, 2)],
                         ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}")
def test_force_matches_oracle(case):
    dims, bc, kappa, eps, n = case
    note(f"force {dims} {bc} n={n}")
    u, lat, d = make(dims, bc, kappa, eps, 1000)
    phi = synth.gaussian_spinors(dims, bc, n, 2000)
    g, action, stats, rc, x, y = lat.force(to_dev(phi), tol=1e-13, prec="fp64", want_xy=True)
    assert rc == 0
    g, x, y = to_host(g), to_host(x), to_host(y)
    # the force kernel alone, fed the same X and Y: FP64 parity at 1e-12
    g_same = fmod.coefficients_to_matrix(fmod.force_coefficients(d, x, y))
    assert rel(g, g_same) < 1e-12
    # links that never enter D hold exactly zero
    from oracle.hmc import entering_mask
    assert not np.any(g[~entering_mask(dims, bc)])
    # the whole chain against the oracle's two solves (Alg. 2)
    g_ref, s_ref, x_ref, y_ref = fmod.fermion_force(d, phi, tol=1e-14)
    c = _cond(d, phi)
    bound = c * 2e-13 + 1e-12
    assert rel(x, x_ref) < bound and rel(y, y_ref) < bound
    assert rel(g, g_ref) < bound
    np.testing.assert_allclose(action, s_ref, rtol=bound)
    lat.close()


_CONFIG1_ORACLE = {}


def _config1_oracle():
    """The oracle's Alg. 2 on the 8^3x8 SF 5-RHS case: X = D^-1 Phi and
    Y = (D^+)^-1 X by per-RHS FP64 CG (the compiled operator) to 1e-13, the
    literal per-generator force and the action (computed once per session)."""
    if not _CONFIG1_ORACLE:
        from oracle import native
        p = synth.CONFIG_1
        u, phi = p.links(), p.rhs()
        nd = native.NativeWilson(p.dims, p.bc, p.kappa, u)
        x, _ = solvers.solve_D(nd, phi, 1e-13)
        y, _ = solvers.solve_Ddag(nd, x, 1e-13)
        g = fmod.coefficients_to_matrix(fmod.force_coefficients(WilsonDirac(p.dims, p.bc, p.kappa, u), x, y))
        _CONFIG1_ORACLE.update(g=g, x=x, y=y, s=fmod.action(None, x))
    return _CONFIG1_ORACLE


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_force_config1_matches_oracle(prec):
    """Summed force, X, Y and the action on the 8^3x8 SF 5-RHS case against the
    oracle's Alg. 2: mixed-precision solves to 1e-12 give forces within 1e-8
    and solutions within 1e-9; the FP64 path, solved to 1e-13, is within
    1e-10 (the solution error is bounded by cond(D^+D) times the residual)."""
    p = synth.CONFIG_1
    ref = _config1_oracle()
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(p.links()))
    tol = 1e-13 if prec == "fp64" else 1e-12
    g, a, stats, rc, x, y = lat.force(to_dev(p.rhs()), tol=tol, prec=prec, want_xy=True)
    assert rc == 0
    eg, ex, ey = rel(to_host(g), ref["g"]), rel(to_host(x), ref["x"]), rel(to_host(y), ref["y"])
    note(f"force {prec} vs oracle: G {eg:.2e} X {ex:.2e} Y {ey:.2e}, iters {[s['iters'] for s in stats]}")
    bound_f, bound_x = (1e-10, 1e-10) if prec == "fp64" else (1e-8, 1e-9)
    assert eg < bound_f and ex < bound_x and ey < bound_x
    np.testing.assert_allclose(a, ref["s"], rtol=bound_x)
    lat.close()
