"""Pins for the oracle's Chebyshev bandpass filters and power spectra (section 2, Eq. 4)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from scipy import integrate

from oracle import chebyshev as ch
from oracle import dense, lattice
from paper_2112_04556_amd import inputs


@pytest.mark.parametrize("lo,hi", [(0.0, 1.0), (3.0, 5.5), (15.0, 16.0), (7.9, 8.1)])
def test_indicator_coefficients_by_quadrature(lo, hi):
    """c_k = (2 - delta_k0)/pi int_{x_lo}^{x_hi} T_k(x) / sqrt(1 - x^2) dx, by adaptive quadrature."""
    D = 12
    c = ch.indicator_coefficients([lo, hi], D)[0]
    xlo, xhi = lo / 8 - 1, hi / 8 - 1
    for k in range(D + 1):
        Tk = npcheb.Chebyshev.basis(k)
        # substitute x = -cos(u) near the ends to tame the 1/sqrt singularity
        val, _ = integrate.quad(lambda u: Tk(-np.cos(u)), np.arccos(-xlo), np.arccos(-xhi),
                                epsabs=1e-14, epsrel=1e-13, limit=200)
        ref = (2 - (k == 0)) / np.pi * val
        assert abs(c[k] - ref) < 1e-12


def test_jackson_matches_autocorrelation():
    """The Jackson factors are the normalised autocorrelation of a_j = sin(pi (j+1)/(N+1))."""
    for D in (8, 64, 255):
        N = D + 1
        a = np.sin(np.pi * (np.arange(N) + 1) / (N + 1))
        auto = np.array([np.dot(a[:N - k], a[k:]) for k in range(N)]) / np.dot(a, a)
        assert np.allclose(ch.jackson(D), auto, atol=1e-13)


@pytest.mark.parametrize("D,nw", [(64, 16), (256, 64), (256, 128)])
def test_partition_of_unity(D, nw):
    coef = ch.window_coefficients(ch.equal_windows(nw), D)
    s = coef.sum(axis=0)
    e0 = np.zeros(D + 1)
    e0[0] = 1
    assert np.abs(s - e0).max() < 1e-13


def test_jackson_windows_nonnegative():
    coef = ch.window_coefficients(ch.equal_windows(16), 64)
    lam = np.linspace(0, 16, 4001)
    p = ch.window_polynomial(coef, lam)
    assert p.min() > -1e-12
    raw = ch.window_polynomial(ch.window_coefficients(ch.equal_windows(16), 64, "none"), lam)
    assert raw.min() < -0.05          # undamped windows ring (Gibbs)


def _dense_setup(L, kind="eps", seed=1):
    U = inputs.random_links(L, kind, 0.5, seed=seed).numpy()
    w, Q = dense.eigh(dense.dense_laplacian(U, L))
    return U, w, Q


def test_recursion_matches_cosines_on_eigenvalues():
    L = (2, 2, 2, 2)
    U, w, Q = _dense_setup(L)
    F = inputs.gaussian_fields(L, 2, seed=3).numpy()
    D = 20
    mu = ch.moments(U, F, L, D)
    V = lattice.volume(L)
    # project each nu block on the eigenbasis: mu_k = sum_i |<e_i, F>|^2 cos(k arccos x_i)
    amp = np.einsum("ji,nqj->nqi", Q, F.reshape(2, 4, 8 * V)) ** 2
    x = np.clip(w / 8 - 1, -1, 1)
    Tk = np.cos(np.outer(np.arange(D + 1), np.arccos(x)))
    ref = np.einsum("nqi,ki->nk", amp, Tk)
    assert np.allclose(mu, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    assert np.all(np.abs(mu) <= mu[:, :1] * (1 + 1e-12))


def test_power_spectrum_dense():
    L = (2, 2, 2, 2)
    U, w, Q = _dense_setup(L, "haar", 5)
    F = inputs.gaussian_fields(L, 1, seed=6).numpy()
    D, nw = 32, 8
    edges = ch.equal_windows(nw)
    mu, pw = ch.power_spectrum(U, F, L, D, edges)
    coef = ch.window_coefficients(edges, D)
    amp = (Q.T @ F.reshape(4, -1).T) ** 2       # (8V, 4)
    ref = ch.window_polynomial(coef, w) @ amp.sum(axis=1)
    assert np.allclose(pw[0], ref, atol=1e-11 * abs(ref).max())
    assert abs(pw.sum() - mu[0, 0]) < 1e-11 * mu[0, 0]     # partition of unity


def test_cheb_filter_dense_and_sum():
    L = (2, 2, 2, 2)
    U, w, Q = _dense_setup(L, "eps", 7)
    x = inputs.gaussian_fields(L, 1, seed=8).numpy()
    D, nw = 24, 4
    edges = ch.equal_windows(nw)
    y = ch.cheb_filter(U, x, L, D, edges)
    coef = ch.window_coefficients(edges, D)
    pw = ch.window_polynomial(coef, w)                       # (nw, 8V)
    for wi in range(nw):
        B = (Q * pw[wi]) @ Q.T
        ref = dense.apply_dense_to_link_field(B, x)
        assert np.allclose(y[wi], ref, atol=1e-12)
    assert np.allclose(y.sum(axis=0), x, atol=1e-12)


def test_free_trace_moments():
    L = (2, 2, 2, 2)
    U = inputs.random_links(L, "unit").numpy()
    w, _ = dense.eigh(dense.dense_laplacian(U, L))
    D = 16
    assert np.allclose(ch.trace_moments_free(L, D), ch.trace_moments_dense(w, D), atol=1e-10)
    den = ch.window_coefficients(ch.equal_windows(16), D) @ ch.trace_moments_free(L, D)
    assert abs(den.sum() - 32 * lattice.volume(L)) < 1e-9


def test_free_moments_by_fft():
    """At U = 1 on an anisotropic lattice: mu_k = sum_p |F(p)|^2 T_k(lambda_p/8 - 1) / V."""
    L = (4, 6, 2, 8)
    U = inputs.random_links(L, "unit").numpy()
    F = inputs.gaussian_fields(L, 1, seed=9).numpy()
    D = 10
    mu = ch.moments(U, F, L, D)[0]
    shp = lattice.lattice_shape(L)
    Fh = np.fft.fftn(F[0].reshape(4, 8, *shp), axes=(2, 3, 4, 5))
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in shp], indexing="ij")
    lam = sum(4 * np.sin(k / 2) ** 2 for k in ks)
    pw = (np.abs(Fh) ** 2).sum(axis=(0, 1)) / lattice.volume(L)
    x = np.arccos(np.clip(lam / 8 - 1, -1, 1))
    ref = np.array([(pw * np.cos(k * x)).sum() for k in range(D + 1)])
    assert np.allclose(mu, ref, atol=1e-10 * ref[0])


def test_free_moments_fft_matches_recursion():
    L = (4, 6, 2, 8)
    U = inputs.random_links(L, "unit").numpy()
    F = inputs.gaussian_fields(L, 2, seed=10).numpy()
    D = 12
    ref = ch.moments(U, F, L, D)
    assert np.allclose(ch.free_moments_fft(F, L, D), ref, atol=1e-10 * ref[:, :1].max())
