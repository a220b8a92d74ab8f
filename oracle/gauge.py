"""Wilson plaquette action and its gauge force (oracle; test infrastructure only).

Section 2 measures power spectra of gauge forces (Fig. 1: Wilson and DBW2 actions).  The Wilson
action is

    S_W = beta sum_x sum_{mu < nu} (1 - Re Tr U_{mu nu}(x) / 3),
    U_{mu nu}(x) = U_mu(x) U_nu(x + mu) U_mu(x + nu)^dag U_nu(x)^dag,

and with the left-multiplication derivative of section 2, U_mu(x) -> exp(i omega^c T^c) U_mu(x),
every plaquette through the link contributes Re Tr(i T^c U_mu(x) S) for its staple S, so

    dS_W / d omega^c_mu(x) = (beta / 3) Im Tr(T^c U_mu(x) A_mu(x)),
    A_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                              + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)].

The gauge force is F_G = -dS_W/d omega (components c = 0..7 of the Gell-Mann basis, as every
link field here).  Everything is literal 3x3 products on numpy arrays with periodic shifts.
"""
from __future__ import annotations

import numpy as np

from . import su3
from .lattice import lattice_shape, shift


def _links(U, L):
    return np.asarray(U).reshape((4,) + lattice_shape(L) + (3, 3))


def _sh(A, mu, sign):
    return shift(A, mu, sign, 0)


def plaquette_traces(U, L) -> np.ndarray:
    """Re Tr U_{mu nu}(x) for the 6 planes mu < nu: shape (6, V)."""
    Ul = _links(U, L)
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = Ul[mu] @ _sh(Ul[nu], mu, +1) @ su3.dagger(_sh(Ul[mu], nu, +1)) @ su3.dagger(Ul[nu])
            out.append(np.trace(P, axis1=-2, axis2=-1).real.reshape(-1))
    return np.stack(out)


def wilson_action(U, L, beta: float) -> float:
    return float(beta * np.sum(1.0 - plaquette_traces(U, L) / 3.0))


def staples(U, L) -> np.ndarray:
    """A_mu(x), shape (4, V, 3, 3)."""
    Ul = _links(U, L)
    out = np.zeros_like(Ul)
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            up = _sh(Ul[nu], mu, +1) @ su3.dagger(_sh(Ul[mu], nu, +1)) @ su3.dagger(Ul[nu])
            down = (su3.dagger(_sh(_sh(Ul[nu], mu, +1), nu, -1)) @ su3.dagger(_sh(Ul[mu], nu, -1))
                    @ _sh(Ul[nu], nu, -1))
            out[mu] += up + down
    return out.reshape(4, -1, 3, 3)


def action_gradient(U, L, beta: float) -> np.ndarray:
    """dS_W / d omega^c_mu(x): shape (4, 8, V)."""
    M = np.asarray(U) @ staples(U, L)                                   # (4, V, 3, 3)
    return (beta / 3.0) * np.einsum("cij,mxji->mcx", su3.T, M).imag


def gauge_force(U, L, beta: float) -> np.ndarray:
    """F_G = -dS_W / d omega, shape (4, 8, V)."""
    return -action_gradient(U, L, beta)


def gauge_force_at(U, L, beta: float, sites) -> np.ndarray:
    """F_G at the given flat site indices only (the definition of ``gauge_force``, the six staples
    of each link formed from its neighbours, for lattices too large for the whole-field version).

    U: (4, V, 3, 3).  Returns (4, 8, len(sites)).
    """
    U = np.asarray(U)
    sites = np.asarray(sites, dtype=np.int64)
    stride = [1, L[0], L[0] * L[1], L[0] * L[1] * L[2]]
    c = np.stack([(sites // stride[mu]) % L[mu] for mu in range(4)], axis=1)

    def at(steps):                       # flat index of x + sum of (direction, sign) steps
        d = c.copy()
        for mu, sign in steps:
            d[:, mu] = (d[:, mu] + sign) % L[mu]
        return d[:, 0] + L[0] * (d[:, 1] + L[1] * (d[:, 2] + L[2] * d[:, 3]))

    out = np.zeros((4, 8, len(sites)))
    for mu in range(4):
        A = np.zeros((len(sites), 3, 3), dtype=np.complex128)
        for nu in range(4):
            if nu == mu:
                continue
            up = U[nu][at([(mu, 1)])] @ su3.dagger(U[mu][at([(nu, 1)])]) @ su3.dagger(U[nu][sites])
            down = (su3.dagger(U[nu][at([(mu, 1), (nu, -1)])]) @ su3.dagger(U[mu][at([(nu, -1)])])
                    @ U[nu][at([(nu, -1)])])
            A += up + down
        M = U[mu][sites] @ A
        out[mu] = -(beta / 3.0) * np.einsum("cij,xji->cx", su3.T, M).imag
    return out

