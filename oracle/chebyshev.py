"""Chebyshev bandpass filters and power spectra (oracle; test infrastructure only).

Section 2 builds a bandpass B(lambda) ~ P_{lambda, dlambda}[-nabla^2_G/16] as a
sum of Chebyshev polynomials and measures the power per mode of a force F as
<F|B|F> / Tr B (Eq. 4).  Readings (listed in the design doc):

* the Chebyshev argument is the affine map of the spectrum [0, 16] onto [-1, 1],
  A = Delta/8 - 1 (the printed argument -nabla^2_G/16 only covers [0, 1]);
* the coefficients are the exact Chebyshev coefficients of the window
  indicator, damped by the Jackson kernel (``kernel="none"`` leaves them undamped);
* "degree D" means T_0 .. T_D; windows are given in Delta units;
* Tr B is the trace over the link-field space (dimension 32 V).

The polynomial T_k(A) x is produced by the plain three-term recursion, one
application of Delta per degree; nothing is blocked or reordered.
"""
from __future__ import annotations

import numpy as np

from .laplacian import laplacian


def equal_windows(n_windows: int, lo: float = 0.0, hi: float = 16.0) -> np.ndarray:
    """n_windows + 1 equally spaced window edges in Delta units."""
    return np.linspace(lo, hi, n_windows + 1)


def indicator_coefficients(edges, degree: int) -> np.ndarray:
    """c[w, k], k = 0..degree: Chebyshev coefficients of the indicator of window w.

    With x = lambda/8 - 1 and theta = arccos x, the indicator of [x_lo, x_hi] has
    c_0 = (theta_lo - theta_hi)/pi and c_k = 2 (sin k theta_lo - sin k theta_hi)/(k pi).
    """
    edges = np.asarray(edges, dtype=np.float64)
    x = np.clip(edges / 8.0 - 1.0, -1.0, 1.0)
    th = np.arccos(x)
    th_lo, th_hi = th[:-1], th[1:]
    k = np.arange(1, degree + 1, dtype=np.float64)
    c = np.empty((len(edges) - 1, degree + 1))
    c[:, 0] = (th_lo - th_hi) / np.pi
    c[:, 1:] = 2.0 * (np.sin(np.outer(th_lo, k)) - np.sin(np.outer(th_hi, k))) / (k * np.pi)
    return c


def jackson(degree: int) -> np.ndarray:
    """Jackson damping factors g_k, k = 0..degree, for N = degree + 1 moments.

    g_k = [(N - k + 1) cos(pi k/(N+1)) + sin(pi k/(N+1)) cot(pi/(N+1))] / (N + 1)
    (the kernel polynomial method of Weisse, Wellein, Alvermann and Fehske, 2006).
    """
    N = degree + 1
    k = np.arange(degree + 1, dtype=np.float64)
    q = np.pi / (N + 1)
    return ((N - k + 1) * np.cos(q * k) + np.sin(q * k) / np.tan(q)) / (N + 1)


def window_coefficients(edges, degree: int, kernel: str = "jackson") -> np.ndarray:
    """coef[w, k] = g_k c[w, k] so that p_w(lambda) = sum_k coef[w, k] T_k(lambda/8 - 1)."""
    c = indicator_coefficients(edges, degree)
    if kernel == "jackson":
        return c * jackson(degree)[None, :]
    if kernel == "none":
        return c
    raise ValueError(kernel)


def window_polynomial(coef: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """p_w(lambda) evaluated with T_k(x) = cos(k arccos x); shape (n_windows, len(lam))."""
    x = np.clip(np.asarray(lam, np.float64) / 8.0 - 1.0, -1.0, 1.0)
    k = np.arange(coef.shape[1])
    Tk = np.cos(np.outer(k, np.arccos(x)))
    return coef @ Tk


def chebyshev_vectors(U, x, L, degree: int):
    """Yield t_k = T_k(A) x for k = 0..degree with A = Delta/8 - 1.

    t_0 = x, t_1 = A x, t_{k+1} = 2 A t_k - t_{k-1}.
    """
    def A(v):
        return laplacian(U, v, L) / 8.0 - v

    t_prev = np.asarray(x, np.float64)
    yield t_prev
    if degree == 0:
        return
    t = A(t_prev)
    yield t
    for _ in range(2, degree + 1):
        t_prev, t = t, 2.0 * A(t) - t_prev
        yield t


def moments(U, F, L, degree: int) -> np.ndarray:
    """mu[n, k] = <F_n, T_k(A) F_n>, summed over nu, for F of shape (n, 4, 8, V)."""
    F = np.asarray(F, np.float64)
    mu = np.empty((F.shape[0], degree + 1))
    for k, t in enumerate(chebyshev_vectors(U, F, L, degree)):
        mu[:, k] = np.sum((F * t).reshape(F.shape[0], -1), axis=1)
    return mu


def power_spectrum(U, F, L, degree: int, edges, kernel: str = "jackson"):
    """(moments[n, k], power[n, w]) with power = <F, p_w(Delta) F>, the numerator of Eq. 4."""
    mu = moments(U, F, L, degree)
    coef = window_coefficients(edges, degree, kernel)
    return mu, mu @ coef.T


def cheb_filter(U, x, L, degree: int, edges, kernel: str = "jackson") -> np.ndarray:
    """y[w] = p_w(Delta) x; shape (n_windows,) + x.shape."""
    coef = window_coefficients(edges, degree, kernel)
    x = np.asarray(x, np.float64)
    y = np.zeros((coef.shape[0],) + x.shape)
    for k, t in enumerate(chebyshev_vectors(U, x, L, degree)):
        y += coef[:, k].reshape((-1,) + (1,) * x.ndim) * t[None]
    return y


def free_spectrum(L) -> np.ndarray:
    """Eigenvalues of Delta at U = 1 on one su(3) colour component: 4 sum_mu sin^2(p_mu/2)."""
    ps = [2.0 * np.pi * np.arange(L[mu]) / L[mu] for mu in range(4)]
    grids = np.meshgrid(*ps, indexing="ij")
    return sum(4.0 * np.sin(g / 2.0) ** 2 for g in grids).ravel()


def trace_moments_free(L, degree: int) -> np.ndarray:
    """Tr T_k(A) over the link-field space (8 colours x 4 directions) at U = 1."""
    lam = free_spectrum(L)
    x = np.clip(lam / 8.0 - 1.0, -1.0, 1.0)
    k = np.arange(degree + 1)
    return 32.0 * np.cos(np.outer(k, np.arccos(x))).sum(axis=1)


def trace_moments_dense(eigenvalues: np.ndarray, degree: int) -> np.ndarray:
    """Tr T_k(A) from the eigenvalues of Delta on one su(3) site field, times 4 directions."""
    x = np.clip(np.asarray(eigenvalues) / 8.0 - 1.0, -1.0, 1.0)
    k = np.arange(degree + 1)
    return 4.0 * np.cos(np.outer(k, np.arccos(x))).sum(axis=1)


def free_moments_fft(F, L, degree: int) -> np.ndarray:
    """mu[n, k] at U = 1 from the plane-wave decomposition: Delta is diagonal in momentum space with
    eigenvalue 4 sum_mu sin^2(p_mu/2) on every colour and direction, so
    mu_k = sum_p |F(p)|^2 T_k(lambda_p/8 - 1) / V (Parseval).  F: (n, 4, 8, V)."""
    F = np.asarray(F, np.float64)
    shp = (int(L[3]), int(L[2]), int(L[1]), int(L[0]))
    V = F.shape[-1]
    ks = np.meshgrid(*[2.0 * np.pi * np.fft.fftfreq(m) for m in shp], indexing="ij")
    lam = sum(4.0 * np.sin(k / 2.0) ** 2 for k in ks)
    th = np.arccos(np.clip(lam / 8.0 - 1.0, -1.0, 1.0)).ravel()
    Tk = np.cos(np.outer(np.arange(degree + 1), th))      # T_k(lambda_p/8 - 1), shared by every field
    mu = np.empty((F.shape[0], degree + 1))
    for i in range(F.shape[0]):
        Fh = np.fft.fftn(F[i].reshape((4, 8) + shp), axes=(2, 3, 4, 5))
        pw = ((np.abs(Fh) ** 2).sum(axis=(0, 1)) / V).ravel()
        mu[i] = Tk @ pw
    return mu
