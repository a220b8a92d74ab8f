"""Link derivatives of the kinetic energy and of R(Delta) (oracle; test infrastructure only).

Section 3 names the extra force from the link dependence of the mass term,
F_M = -Tr{P^dag [d M^{-1}/d U] P}, with d/dU the left-multiplication derivative
of section 2: U_mu(x) -> exp(i omega^c T^c) U_mu(x).  For y = R(Delta[U]) x and a
cotangent g,

    d <g, y> = - sum_j r_j <z_j, (d Delta) x_j>,   x_j = (Delta + sigma_j)^{-1} x,
                                                  z_j = (Delta + sigma_j)^{-1} g,

because d (Delta + sigma)^{-1} = -(Delta + sigma)^{-1} (d Delta) (Delta + sigma)^{-1}
and Delta is self-adjoint.  The kinetic energy K = 1/2 <Y, Y>, Y = R(Delta) P,
has dK = <Y, dY>, i.e. g = Y.  The force is F_M = -dK/d omega.
"""
from __future__ import annotations

import numpy as np

from .laplacian import bilinear_link_derivative
from .rational import shifted_solves


def rational_vjp_links(U, x, g, L, c, r, sigma, tol: float = 1e-13) -> np.ndarray:
    """d <g, R(Delta[U]) x> / d omega, shape (4, 8, V); x, g of shape (n, 4, 8, V), summed over n."""
    x = np.asarray(x, np.float64)
    g = np.asarray(g, np.float64)
    out = np.zeros((4, 8, x.shape[-1]))
    for xi, gi in zip(x, g):
        xs = shifted_solves(U, xi, L, sigma, tol)
        zs = shifted_solves(U, gi, L, sigma, tol)
        for rj, xj, zj in zip(r, xs, zs):
            out -= rj * bilinear_link_derivative(U, zj, xj, L)
    return out


def kinetic_force_grad(U, P, L, c, r, sigma, tol: float = 1e-13) -> np.ndarray:
    """dK/d omega for K = 1/2 sum_n <Y_n, Y_n>, Y = R(Delta) P; shape (4, 8, V)."""
    from .rational import rational_apply
    Y, _ = rational_apply(U, P, L, c, r, sigma, tol)
    return rational_vjp_links(U, P, Y, L, c, r, sigma, tol)
