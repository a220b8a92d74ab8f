"""Periodic 4D lattice geometry (oracle; test infrastructure only).

The paper is silent on boundary conditions; its plane-wave language (section 1)
implies a torus.  Reading: periodic in all four directions, site index
s = x0 + L0*(x1 + L1*(x2 + L2*x3)) with x0 fastest.  A flat site axis of length
V therefore reshapes (C order) to (L3, L2, L1, L0), and direction mu lives on
axis 3 - mu of that block.
"""
from __future__ import annotations

import numpy as np


def volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def lattice_shape(L) -> tuple:
    """(L3, L2, L1, L0): the C-order shape of the flat site index."""
    return (int(L[3]), int(L[2]), int(L[1]), int(L[0]))


def shift(a: np.ndarray, mu: int, sign: int, site_axis: int) -> np.ndarray:
    """b(x) = a(x + sign*mu) on a periodic lattice.

    ``site_axis`` is the first of the four lattice axes (L3, L2, L1, L0) of a.
    """
    return np.roll(a, -sign, axis=site_axis + 3 - mu)


def coords(L) -> np.ndarray:
    """Coordinates (V, 4) of every site, column mu = x_mu."""
    V = volume(L)
    s = np.arange(V)
    out = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        out[:, mu] = s % L[mu]
        s = s // L[mu]
    return out


def neighbour_table(L) -> np.ndarray:
    """Flat indices of x + mu (column 2 mu) and x - mu (column 2 mu + 1), brute force."""
    c = coords(L)
    V = volume(L)
    tab = np.empty((V, 8), dtype=np.int64)
    for mu in range(4):
        for k, sign in enumerate((+1, -1)):
            d = c.copy()
            d[:, mu] = (d[:, mu] + sign) % L[mu]
            tab[:, 2 * mu + k] = d[:, 0] + L[0] * (d[:, 1] + L[1] * (d[:, 2] + L[2] * d[:, 3]))
    return tab
