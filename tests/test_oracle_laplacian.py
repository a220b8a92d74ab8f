"""Pins for the oracle's adjoint covariant Laplacian (section 2, Eq. 3), CPU only."""
import os

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import dense, lattice, su3
from oracle import laplacian as lap
from paper_2112_04556_amd import inputs

ANISO = (4, 6, 2, 8)   # anisotropic so a mixed-up axis or direction cannot pass


def _coords(L):
    return lattice.coords(L)


def test_free_field_plane_waves():
    """At U = 1, cos(k.x) T^a is an eigenvector with eigenvalue 4 sum_mu sin^2(k_mu/2)."""
    L = ANISO
    U = inputs.random_links(L, "unit").numpy()
    c = _coords(L)
    rng = np.random.default_rng(0)
    for trial in range(6):
        n = [rng.integers(0, L[mu]) for mu in range(4)]
        k = np.array([2 * np.pi * n[mu] / L[mu] for mu in range(4)])
        wave = np.cos(c @ k + 0.3)
        P = np.zeros((4, 8, lattice.volume(L)))
        a = trial % 8
        nu = trial % 4
        P[nu, a] = wave
        lam = 4 * np.sum(np.sin(k / 2) ** 2)
        assert np.allclose(lap.laplacian(U, P, L), lam * P, atol=1e-12)


def test_free_field_fft_diagonalises():
    L = ANISO
    U = inputs.random_links(L, "unit").numpy()
    P = inputs.gaussian_fields(L, 1, seed=2).numpy()[0]
    shp = lattice.lattice_shape(L)
    Pl = P.reshape(4, 8, *shp)
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in shp], indexing="ij")
    lam = sum(4 * np.sin(k / 2) ** 2 for k in ks)
    ref = np.fft.ifftn(np.fft.fftn(Pl, axes=(2, 3, 4, 5)) * lam, axes=(2, 3, 4, 5)).real
    assert np.allclose(lap.laplacian(U, P, L), ref.reshape(P.shape), atol=1e-12)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_free_field_multiplicities(L, golden_dir):
    tag = "x".join(map(str, L))
    ref = {}
    with open(os.path.join(golden_dir, "free_field_multiplicities.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t, ev, m = line.split()
            if t == tag:
                ref[float(ev)] = int(m)
    U = inputs.random_links(L, "unit").numpy()
    w, _ = dense.eigh(dense.dense_laplacian(U, L))
    vals, counts = np.unique(np.round(w, 9), return_counts=True)
    got = {float(v) + 0.0: int(cn) for v, cn in zip(vals, counts)}
    assert got == {k: 8 * m for k, m in ref.items()}


def test_self_adjoint():
    L = ANISO
    U = inputs.random_links(L, "haar", seed=3).numpy()
    a = inputs.gaussian_fields(L, 1, seed=4).numpy()
    b = inputs.gaussian_fields(L, 1, seed=5).numpy()
    lhs = lap.inner(a, lap.laplacian(U, b, L))
    rhs = lap.inner(lap.laplacian(U, a, L), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("kind", ["eps", "haar"])
def test_gauge_covariance(kind):
    """Delta[U^Omega](Omega phi Omega^dag) = Omega (Delta[U] phi) Omega^dag, U^Omega_mu(x) = Omega(x) U Omega(x+mu)^dag."""
    L = ANISO
    U = inputs.random_links(L, kind, 0.5, seed=6).numpy()
    Om = inputs.gauge_transform(L, seed=6).numpy()
    nb = lattice.neighbour_table(L)
    UO = np.empty_like(U)
    for mu in range(4):
        UO[mu] = Om @ U[mu] @ su3.dagger(Om[nb[:, 2 * mu]])
    P = inputs.gaussian_fields(L, 1, seed=7).numpy()[0]
    M = su3.to_matrix(np.moveaxis(P, -2, -1))
    PO = np.moveaxis(su3.from_matrix(Om @ M @ su3.dagger(Om)), -1, -2)
    lhs = lap.laplacian(UO, PO, L)
    D = su3.to_matrix(np.moveaxis(lap.laplacian(U, P, L), -2, -1))
    rhs = np.moveaxis(su3.from_matrix(Om @ D @ su3.dagger(Om)), -1, -2)
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (2, 3, 2, 4)])
def test_literal_vs_dense_adjoint_form(L):
    U = inputs.random_links(L, "eps", 0.8, seed=8).numpy()
    P = inputs.gaussian_fields(L, 2, seed=9).numpy()
    D = dense.dense_laplacian(U, L)
    assert np.allclose(lap.laplacian(U, P, L), dense.apply_dense_to_link_field(D, P), atol=1e-13)


def test_spectrum_bounds():
    L = (2, 2, 2, 4)
    for kind in ("eps", "haar"):
        U = inputs.random_links(L, kind, 0.5, seed=10).numpy()
        w, _ = dense.eigh(dense.dense_laplacian(U, L))
        assert w.min() >= -1e-12 and w.max() <= 16 + 1e-12


def test_link_field_is_four_site_fields():
    L = (2, 3, 2, 4)
    U = inputs.random_links(L, "eps", 0.4, seed=11).numpy()
    P = inputs.gaussian_fields(L, 1, seed=12).numpy()[0]
    full = lap.laplacian(U, P, L)
    for nu in range(4):
        assert np.array_equal(full[nu], lap.laplacian(U, P[nu], L))


def test_shift_argument():
    L = (2, 3, 2, 4)
    U = inputs.random_links(L, "eps", 0.4, seed=11).numpy()
    P = inputs.gaussian_fields(L, 1, seed=12).numpy()
    assert np.allclose(lap.laplacian(U, P, L, 0.75), lap.laplacian(U, P, L) + 0.75 * P, atol=1e-14)


def test_link_derivative_central_differences():
    L = (2, 3, 2, 4)
    U = inputs.random_links(L, "eps", 0.5, seed=13).numpy()
    a = inputs.gaussian_fields(L, 2, seed=14).numpy()
    b = inputs.gaussian_fields(L, 2, seed=15).numpy()
    G = lap.bilinear_link_derivative(U, a, b, L)
    rng = np.random.default_rng(3)
    h = 1e-5
    for _ in range(8):
        mu, c, s = rng.integers(4), rng.integers(8), rng.integers(lattice.volume(L))

        def F(e):
            U2 = U.copy()
            U2[mu, s] = expm(1j * e * su3.T[c]) @ U[mu, s]
            return lap.inner(a, lap.laplacian(U2, b, L))

        fd = (F(h) - F(-h)) / (2 * h)
        assert abs(fd - G[mu, c, s]) <= 1e-7 * max(1.0, abs(G[mu, c, s]))


def test_laplacian_at_sites_matches_whole_field():
    L = (3, 4, 2, 5)
    U = inputs.random_links(L, "haar", seed=21).numpy()
    P = inputs.gaussian_fields(L, 2, seed=22).numpy()
    sites = np.array([0, 7, 11, 50, lattice.volume(L) - 1])
    full = lap.laplacian(U, P, L, 0.3)
    assert np.allclose(lap.laplacian_at(U, P, L, sites, 0.3), full[..., sites], atol=1e-13)


def _gather_local(U, a, b, L, mu, sites):
    """Inputs of the per-link derivative for links U_mu(sites): values at x and at x + mu."""
    tab = lattice.neighbour_table(L)
    fwd = tab[sites, 2 * mu]
    return U[mu][sites], a[..., sites], a[..., fwd], b[..., sites], b[..., fwd]


def test_link_derivative_local_central_differences():
    # the per-link form pinned to the definition directly: central differences of <a, Delta[U] b>
    L = (3, 2, 2, 4)
    U = inputs.random_links(L, "eps", 0.5, seed=31).numpy()
    a = inputs.gaussian_fields(L, 2, seed=32).numpy()
    b = inputs.gaussian_fields(L, 2, seed=33).numpy()
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(8):
        mu, c, s = int(rng.integers(4)), int(rng.integers(8)), int(rng.integers(lattice.volume(L)))
        G = lap.bilinear_link_derivative_local(*_gather_local(U, a, b, L, mu, np.array([s])))

        def F(e):
            U2 = U.copy()
            U2[mu, s] = expm(1j * e * su3.T[c]) @ U[mu, s]
            return lap.inner(a, lap.laplacian(U2, b, L))

        fd = (F(h) - F(-h)) / (2 * h)
        assert abs(fd - G[c, 0]) <= 1e-7 * max(1.0, abs(G[c, 0]))


def test_link_derivative_local_matches_whole_field():
    L = (3, 4, 2, 5)
    U = inputs.random_links(L, "haar", seed=34).numpy()
    a = inputs.gaussian_fields(L, 3, seed=35).numpy()
    b = inputs.gaussian_fields(L, 3, seed=36).numpy()
    full = lap.bilinear_link_derivative(U, a, b, L)
    sites = np.arange(lattice.volume(L))
    for mu in range(4):
        loc = lap.bilinear_link_derivative_local(*_gather_local(U, a, b, L, mu, sites))
        assert np.abs(loc - full[mu]).max() <= 1e-12 * np.abs(full).max()
