"""The adjoint covariant Laplacian (oracle; test infrastructure only).

Section 2, Eq. 3 defines nabla^2_G phi(x) = sum_mu [U_mu(x) phi(x+mu) U_mu(x)^dag
+ (backward hop) - 2 phi(x)].  Readings (listed in the design doc):

* the backward hop is U_mu(x-mu)^dag phi(x-mu) U_mu(x-mu) (the printed form has
  a second dagger; only this form is gauge covariant and self-adjoint);
* the paper always uses -nabla^2_G (the normalised operator -nabla^2_G/(4d));
  here Delta = -nabla^2_G >= 0, spectrum in [0, 4d] = [0, 16];
* on a link field P_nu(x) (the momentum and force fields of section 3) Delta acts
  on each nu separately.

Everything is literal 3x3 complex matrix products on numpy arrays.
"""
from __future__ import annotations

import numpy as np

from . import su3
from .lattice import lattice_shape, shift

D = 4  # space-time dimensions


def _links_lattice(U: np.ndarray, L) -> np.ndarray:
    """(4, V, 3, 3) -> (4, L3, L2, L1, L0, 3, 3)."""
    return np.asarray(U).reshape((4,) + lattice_shape(L) + (3, 3))


def laplacian_matrices(U: np.ndarray, Phi: np.ndarray, L) -> np.ndarray:
    """Delta acting on matrix-valued site fields Phi of shape (..., V, 3, 3)."""
    Ul = _links_lattice(U, L)
    lead = Phi.shape[:-3]
    P = Phi.reshape(lead + lattice_shape(L) + (3, 3))
    ax = len(lead)
    out = 2.0 * D * P
    for mu in range(4):
        Uf = Ul[mu]                                   # U_mu(x)
        Ub = shift(Ul[mu], mu, -1, 0)                 # U_mu(x - mu)
        out = out - Uf @ shift(P, mu, +1, ax) @ su3.dagger(Uf)
        out = out - su3.dagger(Ub) @ shift(P, mu, -1, ax) @ Ub
    return out.reshape(Phi.shape)


def laplacian(U: np.ndarray, P: np.ndarray, L, shift_: float = 0.0) -> np.ndarray:
    """(Delta + shift) on component fields P of shape (..., 8, V) (e.g. (n, 4, 8, V))."""
    P = np.asarray(P, dtype=np.float64)
    M = su3.to_matrix(np.moveaxis(P, -2, -1))          # (..., V, 3, 3)
    out = su3.from_matrix(laplacian_matrices(U, M, L))  # (..., V, 8)
    out = np.moveaxis(out, -1, -2)
    if shift_ != 0.0:
        out = out + shift_ * P
    return out


def inner(a: np.ndarray, b: np.ndarray) -> float:
    """<a, b> = sum over every component (sites, directions, generators, fields)."""
    return float(np.sum(np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)))


def bilinear_link_derivative(U: np.ndarray, a: np.ndarray, b: np.ndarray, L) -> np.ndarray:
    """d <a, Delta[U] b> / d omega^c_mu(x) for U_mu(x) -> exp(i omega^c T^c) U_mu(x).

    Section 2 fixes the derivative as left multiplication of the link by the
    generators.  The link U = U_mu(x) enters Delta twice (forward hop at x,
    backward hop at x+mu); differentiating U phi U^dag and U^dag phi U gives

        -2i sum_nu Tr(T^c ([U b(x+mu) U^dag, a(x)] + [U a(x+mu) U^dag, b(x)])).

    a, b: component link fields (..., 4, 8, V), summed over the leading axes and
    nu.  Returns (4, 8, V).
    """
    Ul = _links_lattice(U, L)
    lat = lattice_shape(L)
    A = su3.to_matrix(np.moveaxis(np.asarray(a, np.float64), -2, -1))
    B = su3.to_matrix(np.moveaxis(np.asarray(b, np.float64), -2, -1))
    lead = A.shape[:-3]
    A = A.reshape(lead + lat + (3, 3))
    B = B.reshape(lead + lat + (3, 3))
    ax = len(lead)
    sum_axes = tuple(range(len(lead)))
    out = np.empty((4, 8) + lat)
    for mu in range(4):
        Um = Ul[mu]
        Bf = Um @ shift(B, mu, +1, ax) @ su3.dagger(Um)
        Af = Um @ shift(A, mu, +1, ax) @ su3.dagger(Um)
        comm = (Bf @ A - A @ Bf) + (Af @ B - B @ Af)
        comm = comm.sum(axis=sum_axes)                 # (L3, L2, L1, L0, 3, 3)
        tr = np.einsum("cij,...ji->c...", su3.T, comm)  # Tr(T^c comm)
        out[mu] = (-2j * tr).real
    return out.reshape(4, 8, -1)


def laplacian_at(U: np.ndarray, P: np.ndarray, L, sites, shift_: float = 0.0) -> np.ndarray:
    """(Delta + shift) P evaluated only at the given flat site indices (same definition as
    ``laplacian``, one site at a time, for lattices too large for the whole-field version).

    U: (4, V, 3, 3); P: (..., 8, V) component fields.  Returns (..., 8, len(sites)).
    """
    sites = np.asarray(sites, dtype=np.int64)
    stride = [1, L[0], L[0] * L[1], L[0] * L[1] * L[2]]
    c = np.stack([(sites // stride[mu]) % L[mu] for mu in range(4)], axis=1)
    P = np.asarray(P, np.float64)

    def site_shift(mu, sign):
        d = c.copy()
        d[:, mu] = (d[:, mu] + sign) % L[mu]
        return d[:, 0] + L[0] * (d[:, 1] + L[1] * (d[:, 2] + L[2] * d[:, 3]))

    def mats(idx):                       # (..., len, 3, 3)
        return su3.to_matrix(np.moveaxis(P[..., idx], -2, -1))

    out = 2.0 * D * mats(sites)
    for mu in range(4):
        fwd, bwd = site_shift(mu, +1), site_shift(mu, -1)
        Uf = U[mu][sites]
        Ub = U[mu][bwd]
        out = out - Uf @ mats(fwd) @ su3.dagger(Uf)
        out = out - su3.dagger(Ub) @ mats(bwd) @ Ub
    res = np.moveaxis(su3.from_matrix(out), -1, -2)
    if shift_ != 0.0:
        res = res + shift_ * P[..., sites]
    return res


def bilinear_link_derivative_local(U_links: np.ndarray, a_x: np.ndarray, a_xp: np.ndarray, b_x: np.ndarray,
                                   b_xp: np.ndarray) -> np.ndarray:
    """The same derivative for a set of single links, from values next to each link only.

    For m links U_mu(x) (U_links of shape (m, 3, 3)) the derivative d <a, Delta b> / d omega^c_mu(x)
    involves a and b only at x and x + mu (section 2 derivative, the two hops through the link):
    a_x, b_x are the component values at x and a_xp, b_xp those at x + mu, each of shape
    (..., 8, m) with the leading axes (fields, directions nu) summed.  Returns (8, m).
    This is the per-link form of ``bilinear_link_derivative`` for lattices too large for it.
    """
    def mats(p):
        return su3.to_matrix(np.moveaxis(np.asarray(p, np.float64), -2, -1))   # (..., m, 3, 3)

    Um = np.asarray(U_links)
    Ud = su3.dagger(Um)
    A, Ap, B, Bp = mats(a_x), mats(a_xp), mats(b_x), mats(b_xp)
    Bf = Um @ Bp @ Ud
    Af = Um @ Ap @ Ud
    comm = (Bf @ A - A @ Bf) + (Af @ B - B @ Af)
    comm = comm.reshape((-1,) + comm.shape[-3:]).sum(axis=0)                     # (m, 3, 3)
    tr = np.einsum("cij,mji->cm", su3.T, comm)
    return (-2j * tr).real
