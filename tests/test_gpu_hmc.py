"""GPU molecular dynamics against the oracle's leapfrog (oracle/hmc.py):
kinetic energy, momentum kick and link update element by element, whole
trajectories (final U, P and Delta H, in FP64 and with FP32 inner solves),
the dt^2 scaling of Delta H with the GPU's forces, reversibility, and the
Metropolis decision with restoration on rejection."""
import sys

import numpy as np
import pytest

import synth
from oracle import force as fmod
from oracle import hmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1009_5169_amd as mfq  # noqa: E402

DEV = "cuda:0"
TINY = ((2, 2, 2, 4), "sf", 0.12)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def setup(dims, bc, kappa, seed=11, n_rhs=2):
    u = synth.random_links(dims, bc, 0.3, seed)
    phi = synth.gaussian_spinors(dims, bc, n_rhs, seed + 1)
    pa = synth.gaussian_momenta(dims, bc, 4000 + seed) * hmc.entering_mask(dims, bc)[..., None]
    return u, phi, pa


@pytest.mark.parametrize("case", [TINY, ((4, 2, 2, 4), "periodic", 0.11)], ids=["sf", "periodic"])
def test_kinetic_kick_and_link_update(case):
    dims, bc, kappa = case
    u, phi, pa = setup(dims, bc, kappa)
    mask = hmc.entering_mask(dims, bc)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    pm = fmod.coefficients_to_matrix(pa)
    mom = to_dev(pm)
    k = lat.kinetic_energy(mom)
    k_ref = 0.5 * float(np.sum(pa[mask] ** 2))
    assert abs(k - k_ref) < 1e-13 * k_ref
    # the kick: P - eps G on entering links only
    g = fmod.coefficients_to_matrix(np.random.default_rng(1).standard_normal(pa.shape))
    lat.md_momenta(to_dev(g), mom, 0.37)
    want = np.where(mask[..., None, None], pm - 0.37 * g, pm)
    assert np.abs(to_host(mom) - want).max() < 1e-15
    # the link update: exp(i eps P) U with the oracle's eigendecomposition exponential
    links = to_dev(u)
    lat.md_links(to_dev(pm), links, 0.21)
    got = to_host(links)
    want = np.where(mask[..., None, None], hmc._expi(0.21 * pm) @ u, u)
    assert np.abs(got - want).max() < 1e-14
    assert np.array_equal(got[~mask], u[~mask])          # the others stay bitwise
    uu = got @ np.swapaxes(got.conj(), -1, -2)
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(got) - 1).max() < 1e-14
    lat.close()


@pytest.mark.parametrize("prec,route", [("fp64", "full"), ("fp32", "full"), ("fp64", "schur"), ("fp32", "schur")])
def test_trajectory_matches_oracle_leapfrog(prec, route):
    """The GPU leapfrog against the oracle's, with the forces by route F or by
    route S (the paper's D X = Phi, D^+ Y = X through the Schur complement)."""
    dims, bc, kappa = TINY
    u, phi, pa = setup(dims, bc, kappa)
    md = hmc.FermionMD(dims, bc, kappa, phi)
    tau, n = 0.5, 4
    u_ref, p_ref = md.leapfrog(u, pa, tau, n)
    dh_ref = md.hamiltonian(u_ref, p_ref) - md.hamiltonian(u, pa)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    links, mom = to_dev(u), to_dev(fmod.coefficients_to_matrix(pa))
    res, rc = lat.hmc_trajectory(links, mom, to_dev(phi), tau, n, 0.0, tol=1e-13, prec=prec, max_iter=5000,
                                 route=route)
    assert rc == 0 and res["accepted"] == 1 and res["force_evals"] == n + 1
    note(f"trajectory {prec} {route}: dH gpu {res['delta_h']:.10e} oracle {dh_ref:.10e}")
    assert abs(res["delta_h"] - dh_ref) < 1e-7 * abs(dh_ref) + 1e-10
    assert np.abs(to_host(links) - u_ref).max() < 1e-11
    assert np.abs(fmod.matrix_to_coefficients(to_host(mom)) - p_ref).max() < 1e-10
    assert abs(res["action_old"] - md.action(u)) < 1e-11 * md.action(u)
    assert abs(res["kinetic_old"] - 0.5 * np.sum(pa ** 2)) < 1e-12 * res["kinetic_old"]
    lat.close()


def test_delta_h_scales_as_dt_squared_with_gpu_forces_and_reverses():
    dims, bc, kappa = TINY
    u, phi, pa = setup(dims, bc, kappa)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    dh = []
    for n in (4, 8, 16):
        links, mom = to_dev(u), to_dev(fmod.coefficients_to_matrix(pa))
        res, rc = lat.hmc_trajectory(links, mom, to_dev(phi), 0.5, n, 0.0, tol=1e-13, prec="fp64")
        assert rc == 0
        dh.append(res["delta_h"])
    note(f"dH(n = 4, 8, 16) = {dh}")
    assert 3.5 <= dh[0] / dh[1] <= 4.5 and 3.5 <= dh[1] / dh[2] <= 4.5
    # reversibility: integrate, flip P, integrate again: back to U
    links, mom = to_dev(u), to_dev(fmod.coefficients_to_matrix(pa))
    lat.hmc_trajectory(links, mom, to_dev(phi), 0.5, 8, 0.0, tol=1e-13, prec="fp64")
    mom.neg_()
    res, _ = lat.hmc_trajectory(links, mom, to_dev(phi), 0.5, 8, 0.0, tol=1e-13, prec="fp64")
    assert np.abs(to_host(links) - u).max() < 1e-10
    note(f"reverse trajectory dH {res['delta_h']:.3e}")
    lat.close()


def test_metropolis_rejection_restores_the_start():
    """One big leapfrog step (dH of order 10^3): the draw u = 0 accepts (the
    test is log u < -dH), u = 0.999999 rejects, and a rejection restores the
    links, the momenta and the handle's packed links bitwise."""
    dims, bc, kappa = TINY
    u, phi, pa = setup(dims, bc, kappa, seed=21)
    lat = mfq.Lattice(dims, bc, kappa, to_dev(u))
    pm = fmod.coefficients_to_matrix(pa)
    links, mom = to_dev(u), to_dev(pm)
    res, _ = lat.hmc_trajectory(links, mom, to_dev(phi), 1.0, 1, 0.0, tol=1e-13, prec="fp64")
    note(f"one big step: dH = {res['delta_h']:.4e}, accepted {res['accepted']}")
    assert res["accepted"] == 1 and res["delta_h"] > 1e-3
    assert not np.array_equal(to_host(links), u)
    links, mom = to_dev(u), to_dev(pm)
    res2, _ = lat.hmc_trajectory(links, mom, to_dev(phi), 1.0, 1, 0.999999, tol=1e-13, prec="fp64")
    assert res2["accepted"] == 0
    assert res2["delta_h"] == res["delta_h"]
    assert np.array_equal(to_host(links), u) and np.array_equal(to_host(mom), pm)
    # the handle's packed links were restored too: the action equals the start's
    _, act, _, _ = lat.force(to_dev(phi), tol=1e-13, prec="fp64")
    assert abs(sum(act) - res2["action_old"]) < 1e-11 * res2["action_old"]
    lat.close()
