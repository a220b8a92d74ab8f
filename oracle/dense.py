"""Dense operators for tiny lattices (oracle; test infrastructure only).

Builds Delta on one su(3) site field as a dense (8V x 8V) real matrix from the
adjoint matrices R(U) (a formulation independent of the literal 3x3 products in
``laplacian``):

    Delta = 8 I - sum_mu [ R(U_mu(x)) delta_{y, x+mu} + R(U_mu(x-mu))^T delta_{y, x-mu} ],

since U phi U^dag has components R(U) phi and R(U^dag) = R(U)^T.  Component
ordering: index = a * V + s (generator-major), matching the (8, V) field blocks.
"""
from __future__ import annotations

import numpy as np

from .lattice import neighbour_table, volume
from .su3 import adjoint_matrix


def dense_laplacian(U, L) -> np.ndarray:
    V = volume(L)
    nb = neighbour_table(L)
    R = adjoint_matrix(np.asarray(U))          # (4, V, 8, 8)
    D = 8.0 * np.eye(8 * V)
    rows = np.arange(8)[:, None] * V
    cols = np.arange(8)[None, :] * V
    for s in range(V):
        for mu in range(4):
            fwd = nb[s, 2 * mu]
            bwd = nb[s, 2 * mu + 1]
            D[np.ix_(rows[:, 0] + s, cols[0] + fwd)] -= R[mu, s]
            D[np.ix_(rows[:, 0] + s, cols[0] + bwd)] -= R[mu, bwd].T
    return D


def apply_dense_to_link_field(D: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Apply a dense site-field operator to each nu of P (..., 4, 8, V)."""
    P = np.asarray(P, np.float64)
    flat = P.reshape(P.shape[:-2] + (-1,))
    return (flat @ D.T).reshape(P.shape)


def eigh(D: np.ndarray):
    return np.linalg.eigh(0.5 * (D + D.T))
