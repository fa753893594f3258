"""GPU parity of the multi-lattice persistent batch against the oracle and
against one-lattice solves.  Every lattice's solution must meet the tolerance
on the oracle's own FP64 residual, and agree with a single-lattice solve of the
same system within cond * tol."""
import sys

import numpy as np
import pytest

import synth
from oracle import native, solvers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1009_5169_amd as mfq  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def small_batch(seed=5000, n=7):
    """Uneven lattices (three shapes, ragged site counts) with 1..8 RHS."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(4, 4, 4, 4), (6, 6, 6, 6), (4, 4, 4, 8), (8, 4, 2, 6)]
    probs = []
    for i in range(n):
        dims = shapes[i % len(shapes)]
        probs.append(synth.Problem(f"b{i}", dims, "sf", float(rng.uniform(0.12, 0.135)), 0.3,
                                   int(rng.integers(1, 9)), seed + 1 + i, seed + 1000 + 16 * i))
    return probs


@pytest.mark.parametrize("split", [0, 1], ids=["one_thread_per_site", "direction_split"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_batch_matches_oracle_and_single_solves(prec, split):
    """Both forms of the persistent hopping phases (forced): one thread per
    site, and the four directions split over wavefronts in passes."""
    probs = small_batch()
    note(f"batch {prec} split {split}: " + ", ".join(f"{p.dims}x{p.n_rhs}" for p in probs))
    links = [p.links() for p in probs]
    lats = [mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u)) for p, u in zip(probs, links)]
    rhs = [p.rhs() for p in probs]
    batch = mfq.Batch(lats, [p.n_rhs for p in probs], prec=prec)
    batch.set_shape(batch.grid, split)
    assert batch.split == split
    tol = 1e-10
    xs, stats, rc = batch.solve([to_dev(b) for b in rhs], tol=tol, max_iter=5000)
    note(f"grid {batch.grid}, rc {rc}, iters {[[s['iters'] for s in st] for st in stats]}, "
         f"status {[[s['status'] for s in st] for st in stats]}, "
         f"updates {[[s['reliable_updates'] for s in st] for st in stats]}, "
         f"resid {[max(s['true_rel_resid'] for s in st) for st in stats]}")
    if rc != 0:
        for p, lat, b in zip(probs, lats, rhs):
            xi, sti, rci = lat.solve(to_dev(b), tol=tol, prec=prec, max_iter=5000)
            note(f"  single {p.dims} n={p.n_rhs} k={p.kappa:.4f}: rc {rci} iters {[s['iters'] for s in sti]}")
    assert rc == 0
    for p, u, b, x, st, lat in zip(probs, links, rhs, xs, stats, lats):
        x = to_host(x)
        d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
        r = b - d.DdagD(x)
        for i in range(p.n_rhs):
            res = np.linalg.norm(r[i]) / np.linalg.norm(b[i])
            assert res <= 1.05 * tol, (p.name, i, res)
            assert st[i]["status"] == 0 and st[i]["true_rel_resid"] <= tol
        xi, _, rci = lat.solve(to_dev(b), tol=tol, prec=prec)
        c = solvers.cg_cond(d.DdagD, b, 100)
        err = np.linalg.norm(to_host(xi) - x) / np.linalg.norm(x)
        assert err <= 2 * c * tol, (p.name, err, c)
    batch.close()
    for lat in lats:
        lat.close()


def test_batch_workload_shapes_fp32():
    """A subset of the 64-lattice workload (one lattice of each shape 8^4,
    12^4, 16^3x32), FP32 inner with FP64 reliable updates to 1e-10."""
    probs = synth.batch_problems()
    picked = []
    for shape in [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32)]:
        picked.append(next(p for p in probs if p.dims == shape))
    note("workload subset: " + ", ".join(f"{p.dims}x{p.n_rhs} k={p.kappa:.4f}" for p in picked))
    links = [p.links() for p in picked]
    lats = [mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(u)) for p, u in zip(picked, links)]
    rhs = [p.rhs() for p in picked]
    batch = mfq.Batch(lats, [p.n_rhs for p in picked], prec="fp32")
    xs, stats, rc = batch.solve([to_dev(b) for b in rhs], tol=1e-10, max_iter=10000)
    assert rc == 0
    for p, u, b, x in zip(picked, links, rhs, xs):
        x = to_host(x)
        d = native.NativeWilson(p.dims, p.bc, p.kappa, u)
        r = b - d.DdagD(x)
        for i in range(p.n_rhs):
            assert np.linalg.norm(r[i]) / np.linalg.norm(b[i]) <= 1.05e-10
    batch.close()
    for lat in lats:
        lat.close()


def test_batch_rejects_bad_input():
    p = synth.CONFIG_0
    lat = mfq.Lattice(p.dims, p.bc, p.kappa, to_dev(p.links()))
    with pytest.raises(mfq.MfqError):
        mfq.Batch([lat, lat], [1, 1])
    batch = mfq.Batch([lat], [1], prec="fp64")
    b = p.rhs()
    b[0, 0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(mfq.MfqError):
        batch.solve([to_dev(b)], tol=1e-10)
    with pytest.raises(mfq.MfqError):
        batch.solve([to_dev(p.rhs())], tol=1e-10, prec="fp32")
    batch.close()
    lat.close()
