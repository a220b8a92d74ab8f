"""Link derivatives of the Chebyshev power spectrum and filters (oracle; test infrastructure only).

Section 2 measures the power of a force per mode through a polynomial p(A) of A = Delta/8 - 1
(Eq. 4); its derivative with respect to the links (the left-multiplication derivative of
section 2) follows from the derivative of a matrix function.  For the symmetric operator
A = Q diag(a) Q^T the directional derivative of p(A) is (Daleckii-Krein)

    dp(A) = Q (Gamma o (Q^T dA Q)) Q^T,   Gamma_ij = (p(a_i) - p(a_j)) / (a_i - a_j),

with Gamma_ii = p'(a_i).  Hence, for fields l, r on one direction nu,

    d<l, p(A) r> = sum_ij Gamma_ij (Q^T l)_i (Q^T r)_j  q_i^T dA q_j,

and q_i^T dDelta q_j summed against M_ij is the bilinear link derivative of the Laplacian over
the pairs (q_i, sum_j M_ij q_j), dA = dDelta/8.  Everything here is dense: lattices up to a few
hundred sites.  This is the plain definition, independent of any recursion over degrees.

The divided differences of T_k are taken in the form that has no cancellation: with
x = cos t, y = cos u,  (T_k(x) - T_k(y)) / (x - y) = U_{k-1}(cos((t+u)/2)) U_{k-1}(cos((t-u)/2)),
U the Chebyshev polynomials of the second kind (sin(k s)/sin s = U_{k-1}(cos s)).
"""
from __future__ import annotations

import numpy as np

from . import dense
from .chebyshev import window_coefficients
from .laplacian import bilinear_link_derivative
from .lattice import volume


def _cheb_u(kmax: int, c: np.ndarray) -> np.ndarray:
    """U_0 .. U_kmax at c (any shape): shape (kmax + 1,) + c.shape."""
    out = np.empty((kmax + 1,) + c.shape)
    out[0] = 1.0
    if kmax >= 1:
        out[1] = 2.0 * c
    for k in range(2, kmax + 1):
        out[k] = 2.0 * c * out[k - 1] - out[k - 2]
    return out


def divided_differences(beta: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Gamma_ij = (p(a_i) - p(a_j)) / (a_i - a_j) (p'(a_i) on the diagonal) for
    p(a) = sum_k beta_k T_k(a), a in [-1, 1]."""
    a = np.clip(np.asarray(a, np.float64), -1.0, 1.0)
    th = np.arccos(a)
    s = 0.5 * (th[:, None] + th[None, :])
    d = 0.5 * (th[:, None] - th[None, :])
    D = len(beta) - 1
    if D == 0:
        return np.zeros((len(a), len(a)))
    Us = _cheb_u(D - 1, np.cos(s))
    Ud = _cheb_u(D - 1, np.cos(d))
    # k >= 1: beta_k U_{k-1}(cos s) U_{k-1}(cos d)
    return np.einsum("k,kij,kij->ij", np.asarray(beta[1:], np.float64), Us, Ud)


def _spectral(U, L):
    Dm = dense.dense_laplacian(U, L)
    lam, Q = dense.eigh(Dm)
    return lam / 8.0 - 1.0, Q


def poly_link_derivative(U, L, left, right, beta, spec=None) -> np.ndarray:
    """d<left, p(A[U]) right>/d omega^c_mu(x), p = sum_k beta_k T_k, summed over nu and any leading
    axes of left/right (shape (..., 4, 8, V)).  Returns (4, 8, V)."""
    a, Q = spec if spec is not None else _spectral(U, L)
    G = divided_differences(np.asarray(beta, np.float64), a)
    V = volume(L)
    left = np.asarray(left, np.float64).reshape(-1, 4, 8 * V)
    right = np.asarray(right, np.float64).reshape(-1, 4, 8 * V)
    n = Q.shape[0]
    # the pairs (q_i, sum_j M_ij q_j) of every direction nu and field are site fields (8, V); the
    # bilinear derivative sums over all leading axes, so they go in one batch
    As, Bs = [], []
    for m in range(left.shape[0]):
        for nu in range(4):
            M = G * np.outer(Q.T @ left[m, nu], Q.T @ right[m, nu])
            As.append(Q.T.reshape(n, 8, V))                 # q_i
            Bs.append((M @ Q.T).reshape(n, 8, V))           # sum_j M_ij q_j
    return bilinear_link_derivative(U, np.concatenate(As), np.concatenate(Bs), L) / 8.0


def power_spectrum_link_derivative(U, F, L, degree: int, edges, gamma, kernel: str = "jackson",
                                   per_rhs: bool = False) -> np.ndarray:
    """d(sum_{n,w} gamma[n, w] <F_n, p_w(Delta) F_n>)/d omega: (4, 8, V), or (n, 4, 8, V) per source."""
    coef = window_coefficients(edges, degree, kernel)
    F = np.asarray(F, np.float64)
    gamma = np.asarray(gamma, np.float64)
    spec = _spectral(U, L)
    outs = [poly_link_derivative(U, L, F[i], F[i], gamma[i] @ coef, spec) for i in range(F.shape[0])]
    return np.stack(outs) if per_rhs else np.sum(outs, axis=0)


def power_spectrum_source_gradient(U, F, L, degree: int, edges, gamma, kernel: str = "jackson") -> np.ndarray:
    """d(sum_w gamma[n, w] <F_n, p_w F_n>)/dF_n = 2 sum_w gamma[n, w] p_w(Delta) F_n (dense)."""
    coef = window_coefficients(edges, degree, kernel)
    a, Q = _spectral(U, L)
    F = np.asarray(F, np.float64)
    V = volume(L)
    out = np.empty_like(F)
    Tk = np.cos(np.outer(np.arange(degree + 1), np.arccos(np.clip(a, -1, 1))))
    for i in range(F.shape[0]):
        pa = (np.asarray(gamma[i]) @ coef) @ Tk
        for nu in range(4):
            out[i, nu] = (2.0 * Q @ (pa * (Q.T @ F[i, nu].reshape(8 * V)))).reshape(8, V)
    return out


def cheb_filter_vjp(U, x, gy, L, degree: int, edges, kernel: str = "jackson", per_rhs: bool = False):
    """For y_w = p_w(Delta) x and cotangents gy[w] (shape (n_windows,) + x.shape):
    (grad_x = sum_w p_w(Delta) gy_w, grad_omega = d(sum_w <gy_w, y_w>)/d omega)."""
    coef = window_coefficients(edges, degree, kernel)
    a, Q = _spectral(U, L)
    x = np.asarray(x, np.float64)
    gy = np.asarray(gy, np.float64)
    V = volume(L)
    Tk = np.cos(np.outer(np.arange(degree + 1), np.arccos(np.clip(a, -1, 1))))
    grad_x = np.zeros_like(x)
    gom = []
    for i in range(x.shape[0]):
        g = np.zeros((4, 8, V))
        for w in range(coef.shape[0]):
            pa = coef[w] @ Tk
            for nu in range(4):
                grad_x[i, nu] += (Q @ (pa * (Q.T @ gy[w, i, nu].reshape(8 * V)))).reshape(8, V)
            g += poly_link_derivative(U, L, gy[w, i], x[i], coef[w], (a, Q))
        gom.append(g)
    return grad_x, (np.stack(gom) if per_rhs else np.sum(gom, axis=0))
