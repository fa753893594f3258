"""GPU parity of the learned preconditioner and its flexible GMRES solve:
PTC forward against the oracle (same BF16-valued weights), loss and gradient
of the GPU training kernels against the oracle's analytic gradient, FGMRES
solutions against the oracle residual, CG fallback on a bad network, and the
gain of the trained network over GMRES without it."""
import sys

import numpy as np
import pytest

import synth
from oracle import native, ptc, solvers
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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def flat(w1, w2):
    return np.concatenate([w1[:, :, 0].reshape(-1), w2[:, 0, :].reshape(-1)])


def unflat(w):
    w1 = w[: 9 * 8 * 16].reshape(9, 8, 4, 4)[:, :, None]
    w2 = w[9 * 8 * 16:].reshape(9, 8, 4, 4)[:, None]
    return w1, w2


# the last case has 60 sites per parity: the matrix-core kernel's 16-site
# tiles end in a ragged one
CASES = [((4, 4, 4, 4), "sf"), ((6, 2, 4, 6), "periodic"), ((4, 6, 2, 4), "antiperiodic"), ((6, 2, 2, 6), "sf")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[1]}{'x'.join(map(str, c[0]))}")
def test_ptc_forward_matches_oracle(case):
    dims, bc = case
    u = synth.random_links(dims, bc, 0.5, 31)
    lat = mfq.Lattice(dims, bc, 0.12, to_dev(u))
    w1, w2 = ptc.init_weights(7, scale=0.3)
    lat.precond_set_weights(flat(w1, w2))
    wi1, wi2 = unflat(lat.precond_get_weights("inference"))
    # the inference weights are the BF16 roundings of the FP32 master weights
    assert rel(flat(wi1, wi2), flat(w1, w2)) < 5e-3
    tr = ptc.Transport(WilsonDirac(dims, bc, 0.12, u))
    r = synth.gaussian_spinors(dims, bc, 3, 32)
    got = to_host(lat.precond_apply(to_dev(r)))
    want, _ = ptc.forward(tr, wi1, wi2, r)
    assert rel(got, want) < 2e-5, rel(got, want)
    lat.close()


@pytest.mark.parametrize("case", [((4, 4, 2, 6), "sf"), ((4, 2, 2, 6), "sf"), ((2, 4, 2, 4), "antiperiodic")],
                         ids=["sf-full-tiles", "sf-ragged-tile", "antiperiodic"])
def test_ptc_loss_and_gradient_match_oracle(case):
    """The gradients come from the matrix-core kernels (16-site tiles: the
    second case has 20 sites per parity, a ragged last tile)."""
    dims, bc = case
    u = synth.random_links(dims, bc, 0.5, 33)
    lat = mfq.Lattice(dims, bc, 0.12, to_dev(u))
    w1, w2 = ptc.init_weights(8, scale=0.3)
    lat.precond_set_weights(flat(w1, w2))
    wm1, wm2 = unflat(lat.precond_get_weights("master"))
    r = synth.gaussian_spinors(dims, bc, 4, 34)
    e = synth.gaussian_spinors(dims, bc, 4, 35)
    loss, grad = lat.precond_loss_grad(to_dev(r), to_dev(e))
    tr = ptc.Transport(WilsonDirac(dims, bc, 0.12, u))
    loss_ref, g1, g2 = ptc.loss_and_grad(tr, wm1, wm2, r, e)
    note(f"loss gpu {loss:.8f} oracle {loss_ref:.8f}; grad rel err {rel(grad, flat(g1, g2)):.2e}")
    assert abs(loss - loss_ref) < 1e-5 * loss_ref
    assert rel(grad, flat(g1, g2)) < 1e-3
    lat.close()


def _solve_check(lat, d, b, x, tol):
    x = to_host(x)
    r = b - d.DdagD(x)
    for i in range(b.shape[0]):
        assert np.linalg.norm(r[i]) / np.linalg.norm(b[i]) <= 1.05 * tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("precond", ["identity", "ptc"])
def test_fgmres_solution_meets_tolerance(precond, prec):
    """The cycle in FP64, or in FP32 (basis, operator, network in and out)
    with FP64 restarts: the FP64 true residual meets 1e-10 either way."""
    dims, bc, kappa = (4, 4, 4, 8), "sf", 0.13
    u = synth.random_links(dims, bc, 0.3, 1000)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    # an untrained network close to a multiple of the identity (small random
    # paths): GMRES(16) converges with it as with no preconditioner
    lat.precond_init(seed=3, scale=0.02)
    b = synth.gaussian_spinors(dims, bc, 3, 2000)
    x, stats, rc = lat.solve(to_dev(b), tol=1e-10, precond=precond, prec=prec, max_iter=4000)
    note(f"fgmres {precond} {prec}: rc {rc} iters {[s['iters'] for s in stats]} cycles "
         f"{[s['reliable_updates'] for s in stats]}")
    # GMRES(16) converges here on its own: no hand-over to CG
    assert rc == 0 and all(s["status"] == 0 for s in stats), stats
    _solve_check(lat, native.NativeWilson(dims, bc, kappa, u), b, x, 1e-10)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("restart", [5, 32])
def test_fgmres_restart_lengths_meet_tolerance(restart, prec):
    """Restart lengths other than the default: every basis size 1..restart
    of the Gram-Schmidt kernels (up to the largest, 32) runs, and the solution
    meets the tolerance against the oracle's operator.  kappa = 0.11: GMRES(5)
    without a preconditioner converges there (about 0.6 per cycle in the
    oracle's FGMRES), while at 0.13 it stagnates."""
    dims, bc, kappa = (4, 4, 4, 8), "sf", 0.11
    u = synth.random_links(dims, bc, 0.3, 1000)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    b = synth.gaussian_spinors(dims, bc, 2, 2010)
    x, stats, rc = lat.solve(to_dev(b), tol=1e-10, precond="identity", prec=prec, max_iter=4000,
                             restart=restart)
    note(f"fgmres restart {restart} {prec}: rc {rc} iters {[s['iters'] for s in stats]}")
    assert rc == 0 and all(s["status"] == 0 for s in stats), stats
    _solve_check(lat, native.NativeWilson(dims, bc, kappa, u), b, x, 1e-10)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("precond", ["identity", "ptc"])
def test_fgmres_second_gram_schmidt_pass(precond, prec):
    """kappa = 0.002: |kappa H| <= 16 kappa, so D^+D is within 0.07 of the
    identity and A z_j lies within 7 % of the span of the basis; the first
    projection removes more than 99 % of |w|^2 on every step and the second
    Gram-Schmidt pass runs each time.  The solution meets the tolerance
    against the oracle's operator."""
    dims, bc, kappa = (4, 4, 4, 8), "sf", 0.002
    u = synth.random_links(dims, bc, 0.3, 1000)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    lat.precond_init(seed=3, scale=0.02)
    b = synth.gaussian_spinors(dims, bc, 3, 2040)
    x, stats, rc = lat.solve(to_dev(b), tol=1e-10, precond=precond, prec=prec, max_iter=400)
    note(f"fgmres second pass {precond} {prec}: rc {rc} iters {[s['iters'] for s in stats]}")
    assert rc == 0 and all(s["status"] == 0 for s in stats), stats
    _solve_check(lat, native.NativeWilson(dims, bc, kappa, u), b, x, 1e-10)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("precond", ["identity", "ptc"])
def test_fgmres_graph_replays_match_eager(precond, prec):
    """One restart cycle is captured as a graph and replayed for every cycle
    and by later solves on the same handle.  The reductions have a fixed
    order, so the replays give the eager cycle's solution bit for bit: three
    solves in a row (the third with other right-hand sides), each against an
    eager solve of the same system, with eager work and synchronisations in
    between, and every solution against the oracle's operator."""
    dims, bc, kappa = (4, 4, 4, 8), "sf", 0.13
    u = synth.random_links(dims, bc, 0.3, 1000)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    lat.precond_init(seed=3, scale=0.02)
    op = native.NativeWilson(dims, bc, kappa, u)
    bs = [synth.gaussian_spinors(dims, bc, 3, 2000), synth.gaussian_spinors(dims, bc, 3, 2000),
          synth.gaussian_spinors(dims, bc, 3, 2002)]
    for k, b in enumerate(bs):
        xg, sg, rcg = lat.solve(to_dev(b), tol=1e-10, precond=precond, prec=prec, max_iter=4000, use_graph=True)
        xg = to_host(xg)
        xe, se, rce = lat.solve(to_dev(b), tol=1e-10, precond=precond, prec=prec, max_iter=4000, use_graph=False)
        xe = to_host(xe)
        note(f"fgmres graph {precond} {prec} solve {k}: rc {rcg}/{rce} iters {[s['iters'] for s in sg]}")
        assert rcg == 0 and rce == 0, (sg, se)
        assert [s["iters"] for s in sg] == [s["iters"] for s in se]
        assert np.array_equal(xg, xe)
        r = b - op.DdagD(xg)
        for i in range(b.shape[0]):
            assert np.linalg.norm(r[i]) / np.linalg.norm(b[i]) <= 1.05e-10
    lat.close()


def test_bad_network_falls_back_to_cg():
    dims, bc, kappa = (4, 4, 4, 4), "sf", 0.125
    u = synth.random_links(dims, bc, 0.3, 1000)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    rng = np.random.default_rng(0)
    w = (rng.standard_normal(mfq.N_PTC_COMPLEX) + 1j * rng.standard_normal(mfq.N_PTC_COMPLEX)) * 1e3
    w[: 9 * 8 * 16] = 0.0   # layer 1 maps everything to zero: M = 0
    lat.precond_set_weights(w)
    b = synth.gaussian_spinors(dims, bc, 2, 2000)
    x, stats, rc = lat.solve(to_dev(b), tol=1e-10, precond="ptc", prec="fp64", max_iter=2000)
    note(f"fallback: rc {rc} stats {stats}")
    assert rc == 2
    assert all(s["status"] == 2 for s in stats)
    _solve_check(lat, native.NativeWilson(dims, bc, kappa, u), b, x, 1e-10)
    lat.close()


def test_pairs_training_and_gain(tmp_path):
    """Pairs from CG on b = A xi with known solutions xi, GPU training, and the
    gain of the trained network: fewer FGMRES iterations than without the
    network on evaluation RHS disjoint from the training ones."""
    dims, bc, kappa = (8, 8, 8, 8), "sf", 0.1375
    u = synth.random_links(dims, bc, 0.5, 1004)
    d = native.NativeWilson(dims, bc, kappa, u)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    xi = synth.gaussian_spinors(dims, bc, 4, synth.PTC_TRAIN_SEED)
    r, e = lat.precond_pairs(to_dev(xi), every=5, n_snap=4)
    rh, eh = to_host(r), to_host(e)
    assert rh.shape == (16,) + xi.shape[1:]
    # the first pair is (A xi, xi) / |A xi|, against the oracle operator
    axi = d.DdagD(xi)
    scale = np.linalg.norm(axi.reshape(4, -1), axis=1)[:, None, None, None, None, None, None]
    assert rel(rh[:4], axi / scale) < 1e-12
    assert rel(eh[:4], xi / scale) < 1e-12
    # every pair satisfies A e = r (the CG iterates cancel) with |r| = 1
    res = np.linalg.norm(rh - d.DdagD(eh)) / np.linalg.norm(rh)
    assert res < 1e-12, res
    np.testing.assert_allclose(np.linalg.norm(rh.reshape(16, -1), axis=1), 1.0, rtol=1e-12)
    # the second pair is the oracle's CG iterate after 5 iterations on b = A xi
    x5, _ = solvers.cg(d.DdagD, axi, 0.0, max_iter=5)
    r5 = axi - d.DdagD(x5)
    s5 = np.linalg.norm(r5.reshape(4, -1), axis=1)[:, None, None, None, None, None, None]
    assert rel(rh[4:8], r5 / s5) < 1e-10
    assert rel(eh[4:8], (xi - x5) / s5) < 1e-10
    lat.precond_init(seed=1)
    hist = lat.precond_train(r, e, steps=300, lr=3e-3)
    note(f"training loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.5 * hist[0]
    path = str(tmp_path / "w.bin")
    lat.precond_save(path)
    w_trained = lat.precond_get_weights("master")
    b = synth.gaussian_spinors(dims, bc, 3, 2400)
    x_id, st_id, _ = lat.solve(to_dev(b), tol=1e-10, precond="identity", prec="fp64", max_iter=20000)
    x_pc, st_pc, rc = lat.solve(to_dev(b), tol=1e-10, precond="ptc", prec="fp64", max_iter=20000)
    it_id = [s["iters"] for s in st_id]
    it_pc = [s["iters"] for s in st_pc]
    note(f"FGMRES(16) iterations: identity {it_id}, trained PTC {it_pc} (rc {rc})")
    assert rc == 0
    _solve_check(lat, d, b, x_pc, 1e-10)
    assert sum(it_pc) < 0.8 * sum(it_id)
    lat.precond_load(path)
    np.testing.assert_array_equal(lat.precond_get_weights("master"), w_trained)
    lat.close()


def test_adam_kernel_matches_oracle():
    """Three training steps on the GPU from known weights: after each, the FP32
    master weights and Adam's two moment estimates equal the oracle's
    adam_step (FP64, Kingma and Ba's Algorithm 1) applied to the gradient the
    step used (the loss gradient at the weights before it), element by
    element at FP32 tolerance."""
    dims, bc = (4, 4, 2, 6), "sf"
    u = synth.random_links(dims, bc, 0.5, 36)
    lat = mfq.Lattice(dims, bc, 0.12, to_dev(u))
    lat.precond_init(seed=9, scale=0.3)
    r = to_dev(synth.gaussian_spinors(dims, bc, 3, 37))
    e = to_dev(synth.gaussian_spinors(dims, bc, 3, 38))
    lr = 3e-3
    w = lat.precond_get_weights("master")
    assert not np.any(lat.precond_get_weights("adam_m")) and not np.any(lat.precond_get_weights("adam_v"))
    m = v = np.zeros_like(w)
    for t in range(1, 4):
        _, g = lat.precond_loss_grad(r, e)
        lat.precond_train(r, e, steps=1, lr=lr)
        w_ref, m_ref, v_ref = ptc.adam_step(w, g, m, v, t, lr=lr)
        w_gpu = lat.precond_get_weights("master")
        m_gpu = lat.precond_get_weights("adam_m")
        v_gpu = lat.precond_get_weights("adam_v")
        step_err = np.abs(w_gpu - w_ref).max()
        note(f"adam t={t}: max |w_gpu - w_oracle| = {step_err:.2e} (lr {lr}), "
             f"m {rel(m_gpu, m_ref):.2e}, v {rel(v_gpu, v_ref):.2e}")
        # FP32 master weights: one rounding of w (|w| < 1) plus the step's
        assert step_err < 2e-7 + 1e-4 * lr
        np.testing.assert_allclose(m_gpu.real, m_ref.real, rtol=2e-6, atol=1e-7 * np.abs(m_ref).max())
        np.testing.assert_allclose(m_gpu.imag, m_ref.imag, rtol=2e-6, atol=1e-7 * np.abs(m_ref).max())
        np.testing.assert_allclose(v_gpu.real, v_ref.real, rtol=2e-6, atol=1e-7 * np.abs(v_ref).max())
        np.testing.assert_allclose(v_gpu.imag, v_ref.imag, rtol=2e-6, atol=1e-7 * np.abs(v_ref).max())
        # continue from the GPU's FP32 state (the oracle's FP64 state would drift
        # from it by FP32 roundings only)
        w, m, v = w_gpu, m_gpu, v_gpu
    # the inference copy is the BF16 rounding of the master weights
    wi = lat.precond_get_weights("inference")
    assert np.abs(wi.real - w.real).max() <= 2 ** -8 * np.abs(w.real).max()
    lat.close()
