"""Wilson-Dirac operator, FP64, full lattice.  Test infrastructure only.

The paper uses Wilson quarks with hopping parameter kappa (Sections 3.1 and 4)
without writing the operator out.  Reading used here (Wilson parameter r = 1,
no clover term):

    (D psi)(n) = psi(n) - kappa * sum_mu [ (1 - g_mu) U_mu(n) psi(n+mu)
                                          + (1 + g_mu) U_mu(n-mu)^+ psi(n-mu) ]

and its adjoint, coded separately from its own formula,

    (D^+ psi)(n) = psi(n) - kappa * sum_mu [ (1 + g_mu) U_mu(n) psi(n+mu)
                                            + (1 - g_mu) U_mu(n-mu)^+ psi(n-mu) ].

Gamma matrices: chiral basis g_mu = [[0, e_mu], [e_mu^+, 0]] with e_0 = -1 and
e_k = -i sigma_k, so g_5 = g_0 g_1 g_2 g_3 = diag(1, 1, -1, -1).

Time boundaries:
* Schroedinger functional (SF): time slices x0 = 0..T, spinors vanish on
  x0 = 0 and x0 = T (homogeneous boundary values), dynamical slices 1..T-1;
  space periodic.  Hops onto the boundary slices therefore drop out.
* periodic, or antiperiodic in time (sign -1 on hops that wrap in time).

Array conventions are those of the ``synth`` module: links
``[mu][x0][z][y][x][3][3]`` and spinors ``[rhs][t][z][y][x][4][3]``.
"""
from __future__ import annotations

import numpy as np

SF, PERIODIC, ANTIPERIODIC = "sf", "periodic", "antiperiodic"

_SIGMA = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]],
                  dtype=np.complex128)


def gamma_matrices() -> tuple[np.ndarray, np.ndarray]:
    """(g[4], g5): g[0] is the time direction, g[1..3] are x, y, z."""
    e = [-np.eye(2, dtype=np.complex128)] + [-1j * s for s in _SIGMA]
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for mu in range(4):
        g[mu, :2, 2:] = e[mu]
        g[mu, 2:, :2] = e[mu].conj().T
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


GAMMA, GAMMA5 = gamma_matrices()
ONE4 = np.eye(4, dtype=np.complex128)

# axis of direction mu in a full spinor array [rhs][x0][z][y][x][4][3]
_SPINOR_AXIS = {0: 1, 1: 4, 2: 3, 3: 2}


class WilsonDirac:
    """D[U] for one lattice.  dims = (Lx, Ly, Lz, T)."""

    def __init__(self, dims, bc: str, kappa: float, links: np.ndarray):
        self.dims = tuple(int(d) for d in dims)
        self.bc = bc
        self.kappa = float(kappa)
        lx, ly, lz, t = self.dims
        self.n_slices = t + 1 if bc == SF else t       # stored link slices
        self.t_dyn = t - 1 if bc == SF else t          # dynamical slices
        self.t0 = 1 if bc == SF else 0                 # first dynamical x0
        want = (4, self.n_slices, lz, ly, lx, 3, 3)
        if links.shape != want:
            raise ValueError(f"links shape {links.shape}, expected {want}")
        self.U = np.asarray(links, dtype=np.complex128)
        # contiguous U^T and conj(U) so that the colour products below are
        # plain batched matrix products
        self._ut = np.ascontiguousarray(np.swapaxes(self.U, -1, -2))
        self._uc = np.ascontiguousarray(self.U.conj())

    # ---- geometry -------------------------------------------------------
    def spinor_shape(self, n_rhs: int):
        lx, ly, lz, _ = self.dims
        return (n_rhs, self.t_dyn, lz, ly, lx, 4, 3)

    def embed(self, psi: np.ndarray) -> np.ndarray:
        """Dynamical-slice spinor -> array over all link slices (zeros on the
        SF boundary slices)."""
        if self.bc != SF:
            return psi.copy()
        full = np.zeros((psi.shape[0], self.n_slices) + psi.shape[2:], dtype=np.complex128)
        full[:, 1:-1] = psi
        return full

    def restrict(self, full: np.ndarray) -> np.ndarray:
        return full[:, 1:-1].copy() if self.bc == SF else full

    def shift_fwd(self, f: np.ndarray, mu: int) -> np.ndarray:
        """g(n) = f(n + mu) on a full array, with the time boundary rule."""
        ax = _SPINOR_AXIS[mu]
        if mu != 0 or self.bc == PERIODIC:
            return np.roll(f, -1, axis=ax)
        if self.bc == ANTIPERIODIC:
            g = np.roll(f, -1, axis=ax)
            g[:, -1] *= -1.0
            return g
        g = np.zeros_like(f)            # SF: nothing beyond x0 = T
        g[:, :-1] = f[:, 1:]
        return g

    def shift_bwd(self, f: np.ndarray, mu: int) -> np.ndarray:
        """g(n) = f(n - mu) on a full array, with the time boundary rule."""
        ax = _SPINOR_AXIS[mu]
        if mu != 0 or self.bc == PERIODIC:
            return np.roll(f, 1, axis=ax)
        if self.bc == ANTIPERIODIC:
            g = np.roll(f, 1, axis=ax)
            g[:, 0] *= -1.0
            return g
        g = np.zeros_like(f)            # SF: nothing before x0 = 0
        g[:, 1:] = f[:, :-1]
        return g

    # ---- colour products on full arrays -----------------------------------
    def u_times(self, mu: int, f: np.ndarray) -> np.ndarray:
        """(U_mu(n) f(n)) for every n; f is [rhs][x0][z][y][x][4][3]."""
        return f @ self._ut[mu]

    def udag_times(self, mu: int, f: np.ndarray) -> np.ndarray:
        """(U_mu(n)^+ f(n)) for every n."""
        return f @ self._uc[mu]

    # ---- the operator -------------------------------------------------------
    def hop(self, psi: np.ndarray, dagger: bool = False) -> np.ndarray:
        """H psi (dagger=False) or H^+ psi, with D = 1 - kappa H."""
        f = self.embed(psi)
        out = np.zeros_like(f)
        for mu in range(4):
            p_fwd = ONE4 + GAMMA[mu] if dagger else ONE4 - GAMMA[mu]
            p_bwd = ONE4 - GAMMA[mu] if dagger else ONE4 + GAMMA[mu]
            out += p_fwd @ self.u_times(mu, self.shift_fwd(f, mu))
            out += p_bwd @ self.shift_bwd(self.udag_times(mu, f), mu)
        return self.restrict(out)

    def D(self, psi):
        return psi - self.kappa * self.hop(psi, dagger=False)

    def Ddag(self, psi):
        return psi - self.kappa * self.hop(psi, dagger=True)

    def DdagD(self, psi):
        return self.Ddag(self.D(psi))

    def DDdag(self, psi):
        return self.D(self.Ddag(psi))

    def gamma5(self, psi):
        return GAMMA5 @ psi

    # ---- dense form (tiny lattices only) -------------------------------------
    def dense(self, op: str = "D") -> np.ndarray:
        n = int(np.prod(self.spinor_shape(1)))
        f = getattr(self, op)
        m = np.zeros((n, n), dtype=np.complex128)
        chunk = 192
        for j0 in range(0, n, chunk):
            k = min(chunk, n - j0)
            e = np.zeros((k, n), dtype=np.complex128)
            e[np.arange(k), j0 + np.arange(k)] = 1.0     # unit vectors as RHS
            m[:, j0:j0 + k] = f(e.reshape(self.spinor_shape(k))).reshape(k, n).T
        return m


def even_odd_mask(dims, bc: str) -> np.ndarray:
    """Boolean [t][z][y][x] mask of even sites, (x0 + x + y + z) even, over
    the dynamical slices."""
    lx, ly, lz, t = dims
    t0, td = (1, t - 1) if bc == SF else (0, t)
    x0 = np.arange(t0, t0 + td)[:, None, None, None]
    z = np.arange(lz)[None, :, None, None]
    y = np.arange(ly)[None, None, :, None]
    x = np.arange(lx)[None, None, None, :]
    return ((x0 + x + y + z) % 2) == 0
