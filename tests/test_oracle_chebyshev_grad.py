"""Pins for the oracle's link derivatives of the Chebyshev power spectrum and filter (section 2,
Eq. 4), CPU only: the dense spectral formula against finite differences through the three-term
recursion (an independent route), the divided differences against their direct quotient, and
the filter's source gradient against the adjoint identity."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import chebyshev as och
from oracle import chebyshev_grad as ocg
from oracle import lattice, su3
from paper_2112_04556_amd import inputs

L_SMALL = (2, 3, 2, 2)   # 24 sites: dense operator 192 x 192, anisotropic


def _perturb(U, mu, s, c, eps):
    U2 = U.copy()
    U2[mu, s] = expm(1j * eps * su3.T[c]) @ U[mu, s]
    return U2


def test_divided_differences_against_direct_quotient():
    rng = np.random.default_rng(0)
    beta = rng.normal(size=13)
    a = np.sort(rng.uniform(-1, 1, 9))

    def p(x):
        return np.polynomial.chebyshev.chebval(x, beta)

    G = ocg.divided_differences(beta, a)
    for i in range(len(a)):
        for j in range(len(a)):
            if i != j:
                assert abs(G[i, j] - (p(a[i]) - p(a[j])) / (a[i] - a[j])) <= 1e-10 * max(1.0, abs(G[i, j]))
    dp = np.polynomial.chebyshev.chebval(a, np.polynomial.chebyshev.chebder(beta))
    assert np.allclose(np.diag(G), dp, rtol=1e-12, atol=1e-12)
    # end points and coincident values
    e = np.array([-1.0, -1.0, 1.0, 1.0, 0.3, 0.3])
    Ge = ocg.divided_differences(beta, e)
    assert np.allclose(Ge[0, 1], np.polynomial.chebyshev.chebval(-1.0, np.polynomial.chebyshev.chebder(beta)))
    assert np.allclose(Ge[2, 3], np.polynomial.chebyshev.chebval(1.0, np.polynomial.chebyshev.chebder(beta)))


@pytest.mark.parametrize("kind", ["eps", "unit"])
def test_power_spectrum_link_derivative_finite_differences(kind):
    L = L_SMALL
    U = inputs.random_links(L, kind, 0.6, seed=31).numpy()
    F = inputs.gaussian_fields(L, 2, seed=32).numpy()
    edges = och.equal_windows(4)
    degree = 12
    gamma = np.random.default_rng(1).normal(size=(2, 4))
    G = ocg.power_spectrum_link_derivative(U, F, L, degree, edges, gamma)

    def Lfun(Uh):
        _, pw = och.power_spectrum(Uh, F, L, degree, edges)
        return float(np.sum(gamma * pw))

    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(8):
        mu, c, s = rng.integers(4), rng.integers(8), rng.integers(lattice.volume(L))
        fd = (Lfun(_perturb(U, mu, s, c, h)) - Lfun(_perturb(U, mu, s, c, -h))) / (2 * h)
        assert abs(fd - G[mu, c, s]) <= 1e-6 * max(1.0, np.abs(G).max()), (mu, c, s, fd, G[mu, c, s])
    # per-source gradients sum to the total
    Gp = ocg.power_spectrum_link_derivative(U, F, L, degree, edges, gamma, per_rhs=True)
    assert np.allclose(Gp.sum(axis=0), G, atol=1e-12 * np.abs(G).max())


def test_power_spectrum_source_gradient():
    L = L_SMALL
    U = inputs.random_links(L, "haar", seed=33).numpy()
    F = inputs.gaussian_fields(L, 1, seed=34).numpy()
    edges = och.equal_windows(3)
    degree = 10
    gamma = np.array([[0.7, -1.2, 0.4]])
    g = ocg.power_spectrum_source_gradient(U, F, L, degree, edges, gamma)
    # twice the gamma-weighted filter of F, computed by the recursion
    y = och.cheb_filter(U, F, L, degree, edges)
    assert np.allclose(g, 2 * np.tensordot(gamma[0], y, axes=(0, 0)), atol=1e-11)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(4):
        idx = tuple(rng.integers(n) for n in F.shape)
        Fp, Fm = F.copy(), F.copy()
        Fp[idx] += h
        Fm[idx] -= h
        fp = np.sum(gamma * och.power_spectrum(U, Fp, L, degree, edges)[1])
        fm = np.sum(gamma * och.power_spectrum(U, Fm, L, degree, edges)[1])
        assert abs((fp - fm) / (2 * h) - g[idx]) <= 1e-6 * max(1.0, abs(g[idx]))


def test_cheb_filter_vjp():
    L = L_SMALL
    U = inputs.random_links(L, "eps", 0.8, seed=35).numpy()
    x = inputs.gaussian_fields(L, 2, seed=36).numpy()
    edges = np.array([0.0, 3.0, 7.5, 16.0])
    degree = 9
    gy = np.random.default_rng(4).normal(size=(3,) + x.shape)
    gx, gom = ocg.cheb_filter_vjp(U, x, gy, L, degree, edges)
    # grad_x: the adjoint of the (symmetric) filters applied to the cotangents
    y_of_gy = np.stack([och.cheb_filter(U, gy[w], L, degree, edges)[w] for w in range(3)])
    assert np.allclose(gx, y_of_gy.sum(axis=0), atol=1e-11)

    def Lfun(Uh):
        return float(np.sum(gy * och.cheb_filter(Uh, x, L, degree, edges)))

    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(6):
        mu, c, s = rng.integers(4), rng.integers(8), rng.integers(lattice.volume(L))
        fd = (Lfun(_perturb(U, mu, s, c, h)) - Lfun(_perturb(U, mu, s, c, -h))) / (2 * h)
        assert abs(fd - gom[mu, c, s]) <= 1e-6 * max(1.0, np.abs(gom).max())


def test_degree_zero_has_no_link_dependence():
    L = (2, 2, 2, 2)
    U = inputs.random_links(L, "haar", seed=37).numpy()
    F = inputs.gaussian_fields(L, 1, seed=38).numpy()
    G = ocg.power_spectrum_link_derivative(U, F, L, 0, och.equal_windows(2), np.ones((1, 2)))
    assert np.abs(G).max() == 0.0
