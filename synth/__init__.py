"""Seeded synthetic inputs for the many-flavor quark solve.

This module is shared by the FP64 oracle, the tests and the benchmark.  It
draws random numbers and lays them out in the canonical boundary layout; it
holds none of the method's arithmetic (no Dirac operator, no solver, no force).

Canonical layouts (complex128, x fastest):

* links  ``[mu][x0][z][y][x][3][3]`` with mu = 0 (time), 1 (x), 2 (y), 3 (z).
  Schroedinger-functional (SF) lattices store the T+1 time slices x0 = 0..T so
  that the fixed boundary spatial links are representable; periodic and
  time-antiperiodic lattices store T slices.
* spinors ``[rhs][t][z][y][x][spin 4][color 3]`` over the dynamical time slices
  only: x0 = 1..T-1 for SF (T-1 slices), x0 = 0..T-1 otherwise.

The paper's workload (Section 4: a thermalized 16^4 SF configuration at
beta = 4.52, kappa = 0.15805 with five pseudo-fermions) is not available, so
these generators stand in for it with the same lattice shape and RHS count.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Sequence

import numpy as np

BC_SF = "sf"
BC_PERIODIC = "periodic"
BC_ANTIPERIODIC_T = "antiperiodic"
BCS = (BC_SF, BC_PERIODIC, BC_ANTIPERIODIC_T)

GENERATOR_VERSION = 1

# Gell-Mann matrices lambda_1..lambda_8; the generators used to draw links are
# lambda_a / 2.  They are data for the random draw only.
_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7] = np.diag([1, 1, -2]) / math.sqrt(3)


def _check(dims: Sequence[int], bc: str) -> tuple[int, int, int, int]:
    if bc not in BCS:
        raise ValueError(f"unknown boundary condition {bc!r}")
    lx, ly, lz, t = (int(d) for d in dims)
    if min(lx, ly, lz, t) < 2 or any(d % 2 for d in (lx, ly, lz, t)):
        raise ValueError(f"dims must be even and >= 2, got {dims}")
    if bc == BC_SF and t < 3:
        raise ValueError("SF lattices need T >= 3")
    return lx, ly, lz, t


def link_slices(dims: Sequence[int], bc: str) -> int:
    """Number of stored time slices of the link array."""
    t = _check(dims, bc)[3]
    return t + 1 if bc == BC_SF else t


def spinor_slices(dims: Sequence[int], bc: str) -> int:
    """Number of dynamical time slices (those a spinor array stores)."""
    t = _check(dims, bc)[3]
    return t - 1 if bc == BC_SF else t


def link_shape(dims, bc):
    lx, ly, lz, _ = _check(dims, bc)
    return (4, link_slices(dims, bc), lz, ly, lx, 3, 3)


def spinor_shape(dims, bc, n_rhs):
    lx, ly, lz, _ = _check(dims, bc)
    return (int(n_rhs), spinor_slices(dims, bc), lz, ly, lx, 4, 3)


def _expi_herm(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for the su(3) coefficient rows h (H = sum_a h_a lambda_a/2)."""
    herm = np.einsum("na,aij->nij", h, _GELL_MANN / 2)
    w, v = np.linalg.eigh(herm)
    return np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())


_PARALLEL_MIN = 200_000


def _random_su3(rng: np.random.Generator, n: int, eps: float) -> np.ndarray:
    """n matrices exp(i eps H), H = sum_a h_a lambda_a/2, h_a ~ N(0,1).

    The Gaussian draw happens first; for large n the eigendecompositions run
    in threads over chunks (LAPACK releases the GIL).  The result does not
    depend on the number of threads."""
    h = rng.standard_normal((n, 8))
    workers = min(16, os.cpu_count() or 1)
    if n < _PARALLEL_MIN or workers < 2:
        return _expi_herm(h, eps)
    import concurrent.futures
    chunks = np.array_split(h, workers * 4)
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda c: _expi_herm(c, eps), chunks))
    return np.concatenate(parts)


def sf_boundary_links(l: int) -> tuple[np.ndarray, np.ndarray]:
    """Constant diagonal SU(3) spatial links at x0 = 0 and x0 = T (abelian SF
    background at eta = 0).  They never enter the Wilson operator with
    homogeneous spinor boundary values; they are stored for completeness."""
    c0 = np.diag(np.exp(1j * np.pi / (3 * l) * np.array([-1.0, 0.0, 1.0])))
    ct = np.diag(np.exp(1j * np.pi / (3 * l) * np.array([-3.0, 1.0, 2.0])))
    return c0.astype(np.complex128), ct.astype(np.complex128)


def random_links(dims, bc, eps: float, seed: int) -> np.ndarray:
    """Links U = exp(i eps H) with H a Gaussian su(3) element, one per link."""
    shape = link_shape(dims, bc)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(np.prod(shape[:5]))
    u = _random_su3(rng, n, float(eps)).reshape(shape)
    if bc == BC_SF:
        c0, ct = sf_boundary_links(dims[0])
        u[1:, 0] = c0
        u[1:, -1] = ct
        u[0, -1] = np.eye(3)  # U_0(x0 = T) points off the lattice: unused
    return np.ascontiguousarray(u)


def unit_links(dims, bc) -> np.ndarray:
    shape = link_shape(dims, bc)
    u = np.zeros(shape, dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def gaussian_spinors(dims, bc, n_rhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian spinors, Re and Im ~ N(0, 1/2) (E|z|^2 = 1)."""
    shape = spinor_shape(dims, bc, n_rhs)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal(shape + (2,)) * math.sqrt(0.5)
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def random_gauge_transform(dims, bc, seed: int) -> np.ndarray:
    """Haar-random SU(3) matrix per site, shape [x0][z][y][x][3][3] over the
    link slices; equal to 1 on the SF boundary slices x0 = 0 and x0 = T."""
    lx, ly, lz, _ = _check(dims, bc)
    ts = link_slices(dims, bc)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = ts * lz * ly * lx
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    om = q.reshape(ts, lz, ly, lx, 3, 3)
    if bc == BC_SF:
        om[0] = np.eye(3)
        om[-1] = np.eye(3)
    return np.ascontiguousarray(om)


def gaussian_momenta(dims, bc, seed: int) -> np.ndarray:
    """Real Gaussian su(3) coefficients P^a ~ N(0,1), shape [mu][x0][z][y][x][8]."""
    lx, ly, lz, _ = _check(dims, bc)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((4, link_slices(dims, bc), lz, ly, lx, 8))


def gaussian_momentum_matrices(dims, bc, seed: int) -> np.ndarray:
    """The same draw as ``gaussian_momenta`` laid out as Hermitian traceless
    matrices sum_a P^a lambda_a / 2, shape [mu][x0][z][y][x][3][3] (the
    library's momentum layout)."""
    pa = gaussian_momenta(dims, bc, seed)
    return np.ascontiguousarray(np.tensordot(pa, _GELL_MANN / 2, axes=([5], [0])))


@dataclasses.dataclass(frozen=True)
class Problem:
    """One lattice problem: geometry, hopping parameter, link and RHS seeds."""
    name: str
    dims: tuple
    bc: str
    kappa: float
    eps: float
    n_rhs: int
    link_seed: int
    rhs_seed: int

    def links(self) -> np.ndarray:
        return random_links(self.dims, self.bc, self.eps, self.link_seed)

    def rhs(self) -> np.ndarray:
        return gaussian_spinors(self.dims, self.bc, self.n_rhs, self.rhs_seed)


# The five workloads (small parity case, the benchmark case, the paper's
# 16^3x16 shape in half storage, the uneven batch, and the ill-conditioned
# case for the learned preconditioner).
CONFIG_0 = Problem("sf4x4x4x4_k0.125_1rhs", (4, 4, 4, 4), BC_SF, 0.125, 0.3, 1, 1000, 2000)
CONFIG_1 = Problem("sf8x8x8x8_k0.13_5rhs", (8, 8, 8, 8), BC_SF, 0.13, 0.3, 5, 1001, 2100)
CONFIG_2 = Problem("sf16x16x16x16_k0.135_5rhs", (16, 16, 16, 16), BC_SF, 0.135, 0.5, 5, 1002, 2200)
CONFIG_4 = Problem("sf16x16x16x16_k0.1375_5rhs", (16, 16, 16, 16), BC_SF, 0.1375, 0.5, 5, 1004, 2400)
PTC_TRAIN_SEED = 6000


def batch_problems(seed: int = 5000, n: int = 64) -> list[Problem]:
    """The uneven multi-lattice batch: shapes drawn from {8^4, 12^4, 16^3x32},
    1..8 RHS each, kappa uniform in [0.12, 0.135], eps = 0.3, SF."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32)]
    out = []
    for i in range(n):
        dims = shapes[int(rng.integers(0, 3))]
        n_rhs = int(rng.integers(1, 9))
        kappa = float(rng.uniform(0.12, 0.135))
        out.append(Problem(f"batch{i}", dims, BC_SF, kappa, 0.3, n_rhs,
                           seed + 1 + i, seed + 1000 + 16 * i))
    return out
