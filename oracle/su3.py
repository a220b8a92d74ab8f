"""su(3) in the fundamental representation (oracle; test infrastructure only).

The paper works with the adjoint representation of SU(3) (section 2, Eq. 3) and
fixes no basis.  Reading: Hermitian traceless 3x3 matrices in the basis
T^a = lambda^a / 2 (Gell-Mann), Tr(T^a T^b) = delta^{ab}/2,
[T^a, T^b] = i f^{abc} T^c.  An element phi has real components
phi^a = 2 Tr(T^a phi), so <phi, psi> = sum_a phi^a psi^a = 2 Tr(phi psi).
Index a = 0..7 here stands for the Gell-Mann index a+1.
"""
from __future__ import annotations

import numpy as np


def gell_mann() -> np.ndarray:
    """lambda^1 .. lambda^8, shape (8, 3, 3) complex."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1.0
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1.0, -1.0
    lam[3][0, 2] = lam[3][2, 0] = 1.0
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1.0
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1.0 / np.sqrt(3.0)
    lam[7][2, 2] = -2.0 / np.sqrt(3.0)
    return lam


T = gell_mann() / 2.0


def dagger(M: np.ndarray) -> np.ndarray:
    """Hermitian conjugate over the last two axes."""
    return np.conj(np.swapaxes(M, -1, -2))


def to_matrix(phi: np.ndarray) -> np.ndarray:
    """Components (..., 8) -> Hermitian traceless matrices (..., 3, 3)."""
    return np.einsum("...a,aij->...ij", phi.astype(np.complex128), T)


def from_matrix(M: np.ndarray) -> np.ndarray:
    """Matrices (..., 3, 3) -> components 2 Tr(T^a M), real part, (..., 8)."""
    return 2.0 * np.einsum("aij,...ji->...a", T, M).real


def structure_constants() -> np.ndarray:
    """f^{abc} from the commutators: f^{abc} = -2i Tr([T^a, T^b] T^c)."""
    comm = np.einsum("aij,bjk->abik", T, T) - np.einsum("bij,ajk->abik", T, T)
    f = -2j * np.einsum("abik,cki->abc", comm, T)
    assert np.abs(f.imag).max() < 1e-14
    return f.real


def adjoint_matrix(U: np.ndarray) -> np.ndarray:
    """R^{ab}(U) = 2 Tr(T^a U T^b U^dagger), shape (..., 8, 8): U phi U^dag = (R phi)^a T^a."""
    UTb = np.einsum("...ij,bjk,...lk->...bil", U, T, np.conj(U))
    return 2.0 * np.einsum("aji,...bij->...ab", T, UTb).real
