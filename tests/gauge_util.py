"""Gauge-transformation helpers for the covariance pins (test code only)."""
import numpy as np

_AXES = {0: 0, 1: 3, 2: 2, 3: 1}      # site axes of a [x0][z][y][x] field


def rotate_links(u, om, bc):
    """U_mu(n) -> Om(n) U_mu(n) Om(n+mu)^+ ; om is [x0][z][y][x][3][3]."""
    ut = np.empty_like(u)
    for mu in range(4):
        if mu == 0 and bc == "sf":
            om_fwd = np.empty_like(om)
            om_fwd[:-1] = om[1:]
            om_fwd[-1] = np.eye(3)
        else:
            om_fwd = np.roll(om, -1, axis=_AXES[mu])
        ut[mu] = om @ u[mu] @ np.swapaxes(om_fwd.conj(), -1, -2)
    return ut


def dynamical(om, bc):
    return om[1:-1] if bc == "sf" else om


def rotate_spinors(psi, om, bc):
    """psi(n) -> Om(n) psi(n) on the dynamical slices."""
    return np.einsum("tzyxab,rtzyxsb->rtzyxsa", dynamical(om, bc), psi)


def rotate_link_field(g, om):
    """G_mu(n) -> Om(n) G_mu(n) Om(n)^+ (adjoint action at the link's base)."""
    return om[None] @ g @ np.swapaxes(om.conj(), -1, -2)[None]
