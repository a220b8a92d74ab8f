"""Pins for the oracle's rational mass term, solves, kinetic energy and force (section 3, Eq. 5, Eq. 6)."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import dense, force, lattice, su3
from oracle import laplacian as lap
from oracle import rational as ra
from paper_2112_04556_amd import inputs


def test_poles_from_quadratics_match_direct_evaluation():
    a0, a1, b0, b1 = [0.3, -0.2], [1.1, 0.5], [0.02, 0.5], [0.5, 1.6]
    c, r, s = ra.poles_from_quadratics(0.7, a0, a1, b0, b1)
    lam = np.linspace(0, 16, 57)
    direct = 0.7 + sum(ra.quadratic_term(lam, *t) for t in zip(a0, a1, b0, b1))
    assert np.allclose(ra.rational_scalar(lam, c, r, s), direct, rtol=1e-13, atol=1e-14)
    assert np.all(s > 0)


def test_poles_reject_complex_roots():
    with pytest.raises(ValueError):
        ra.poles_from_quadratics(0.0, [1.0], [0.0], [1.0], [0.5])   # b1^2 < 4 b0


@pytest.mark.parametrize("kappa,n,bound", [(0.9, 8, 4e-4), (0.9, 12, 5e-6), (0.9, 16, 5e-8),
                                           (0.5, 8, 3e-7), (0.5, 12, 1e-10)])
def test_kappa_poles_accuracy(kappa, n, bound):
    c, r, s = ra.kappa_poles(kappa, n)
    lam = np.linspace(0, 16, 20001)
    err = np.abs(ra.rational_scalar(lam, c, r, s) ** 2 * (1 - kappa + kappa * lam) - 1)
    assert err.max() < bound
    assert np.all(r > 0) and np.all(s > 0)


def test_eq2_free_plane_wave():
    """At U = 1: Delta R(Delta)^2 on a plane wave gives k^2/(1 - kappa + kappa k^2) (Eq. 2)."""
    L = (4, 6, 2, 8)
    U = inputs.random_links(L, "unit").numpy()
    c_ = lattice.coords(L)
    kappa = 0.5
    c, r, s = ra.kappa_poles(kappa, 12)
    k = np.array([2 * np.pi * 1 / 4, 2 * np.pi * 2 / 6, np.pi, 2 * np.pi * 3 / 8])
    P = np.zeros((1, 4, 8, lattice.volume(L)))
    P[0, 1, 3] = np.cos(c_ @ k)
    y, _ = ra.rational_apply(U, P, L, c, r, s, tol=1e-14)
    y, _ = ra.rational_apply(U, y, L, c, r, s, tol=1e-14)
    z = lap.laplacian(U, y, L)
    k2 = 4 * np.sum(np.sin(k / 2) ** 2)
    assert np.allclose(z, k2 / (1 - kappa + kappa * k2) * P, atol=1e-9)


def _dense(L, kind="eps", seed=1):
    U = inputs.random_links(L, kind, 0.5, seed=seed).numpy()
    return U, dense.dense_laplacian(U, L)


def test_cg_solve_vs_dense():
    L = (2, 2, 2, 2)
    U, D = _dense(L)
    b = inputs.gaussian_fields(L, 1, seed=2).numpy()[0]
    for sigma in (0.1, 1.0, 50.0):
        x, it, res = ra.cg_solve(U, b, L, sigma, tol=1e-13)
        ref = np.linalg.solve(D + sigma * np.eye(D.shape[0]), b.reshape(4, -1).T).T.reshape(b.shape)
        cond = (16 + sigma) / sigma
        assert res <= 1e-13
        assert np.linalg.norm(x - ref) <= 2 * cond * 1e-13 * np.linalg.norm(ref)


def _dense_rational(D, c, r, s):
    w, Q = dense.eigh(D)
    return (Q * ra.rational_scalar(w, c, r, s)) @ Q.T


def test_rational_apply_and_kinetic_energy_vs_dense():
    L = (2, 2, 2, 2)
    U, D = _dense(L, "haar", 3)
    c, r, s = ra.poles_from_quadratics(0.4, [0.3, 0.1], [1.0, 0.2], [0.05, 0.3], [0.6, 1.4])
    P = inputs.gaussian_fields(L, 2, seed=4).numpy()
    y, xp = ra.rational_apply(U, P, L, c, r, s)
    Rm = _dense_rational(D, c, r, s)
    ref = dense.apply_dense_to_link_field(Rm, P)
    assert np.allclose(y, ref, atol=1e-10)
    K, _ = ra.kinetic_energy(U, P, L, c, r, s)
    Kref = 0.5 * np.sum((ref * ref).reshape(ref.shape[0], -1), axis=1)
    assert np.allclose(K, Kref, rtol=1e-11)
    assert np.all(K > 0)
    # pole solutions: (Delta + sigma_j) x_j = P
    for j, sj in enumerate(s):
        res = lap.laplacian(U, xp[:, j], L, sj) - P
        assert np.abs(res).max() < 1e-11


def test_kinetic_energy_gauge_invariant():
    L = (2, 3, 2, 2)
    U = inputs.random_links(L, "eps", 0.5, seed=5).numpy()
    Om = inputs.gauge_transform(L, seed=5).numpy()
    nb = lattice.neighbour_table(L)
    UO = np.stack([Om @ U[mu] @ su3.dagger(Om[nb[:, 2 * mu]]) for mu in range(4)])
    P = inputs.gaussian_fields(L, 1, seed=6).numpy()
    M = su3.to_matrix(np.moveaxis(P, -2, -1))
    PO = np.moveaxis(su3.from_matrix(Om @ M @ su3.dagger(Om)), -1, -2)
    c, r, s = ra.kappa_poles(0.9, 6)
    K1, _ = ra.kinetic_energy(U, P, L, c, r, s)
    K2, _ = ra.kinetic_energy(UO, PO, L, c, r, s)
    assert np.allclose(K1, K2, rtol=1e-11)


def _dense_K(U, P, L, c, r, s):
    """K from dense R-form matrices and dense linear solves, independent of the CG and commutators."""
    D = dense.dense_laplacian(U, L)
    I = np.eye(D.shape[0])
    flat = P.reshape(P.shape[0], 4, -1)
    Y = c * flat + sum(rj * np.linalg.solve(D + sj * I, flat.reshape(-1, flat.shape[-1]).T).T.reshape(flat.shape)
                       for rj, sj in zip(r, s))
    return 0.5 * np.sum(Y * Y)


def test_kinetic_force_vs_dense_finite_differences():
    L = (2, 2, 2, 2)
    U = inputs.random_links(L, "eps", 0.6, seed=7).numpy()
    P = inputs.gaussian_fields(L, 1, seed=8).numpy()
    c, r, s = ra.poles_from_quadratics(0.2, [0.3], [1.0], [0.05], [0.6])
    G = force.kinetic_force_grad(U, P, L, c, r, s)
    rng = np.random.default_rng(4)
    h = 1e-5
    for _ in range(6):
        mu, cc, x = rng.integers(4), rng.integers(8), rng.integers(lattice.volume(L))

        def K(e):
            U2 = U.copy()
            U2[mu, x] = expm(1j * e * su3.T[cc]) @ U[mu, x]
            return _dense_K(U2, P, L, c, r, s)

        fd = (K(h) - K(-h)) / (2 * h)
        assert abs(fd - G[mu, cc, x]) <= 2e-7 * max(1.0, np.abs(G).max())


def test_force_cartan_zero():
    """At U = 1 with P in the Cartan subalgebra (T^3, T^8) every commutator vanishes: force == 0."""
    L = (2, 2, 2, 4)
    U = inputs.random_links(L, "unit").numpy()
    P = inputs.gaussian_fields(L, 1, seed=9).numpy()
    P[:, :, [0, 1, 3, 4, 5, 6]] = 0.0
    c, r, s = ra.kappa_poles(0.9, 4)
    G = force.kinetic_force_grad(U, P, L, c, r, s)
    assert np.all(G == 0.0)


def test_force_gauge_covariant():
    """dK/domega at link (x, mu) rotates with R(Omega(x)) under a gauge transformation."""
    L = (2, 2, 2, 2)
    U = inputs.random_links(L, "eps", 0.5, seed=10).numpy()
    Om = inputs.gauge_transform(L, seed=10).numpy()
    nb = lattice.neighbour_table(L)
    UO = np.stack([Om @ U[mu] @ su3.dagger(Om[nb[:, 2 * mu]]) for mu in range(4)])
    P = inputs.gaussian_fields(L, 1, seed=11).numpy()
    M = su3.to_matrix(np.moveaxis(P, -2, -1))
    PO = np.moveaxis(su3.from_matrix(Om @ M @ su3.dagger(Om)), -1, -2)
    c, r, s = ra.kappa_poles(0.9, 4)
    G = force.kinetic_force_grad(U, P, L, c, r, s)
    GO = force.kinetic_force_grad(UO, PO, L, c, r, s)
    R = su3.adjoint_matrix(Om)                      # (V, 8, 8)
    assert np.allclose(GO, np.einsum("sab,mbs->mas", R, G), atol=1e-10)


@pytest.mark.parametrize("kappa,n", [(0.5, 12), (0.9, 16)])
def test_heatbath_momenta_against_exact_square_root(kappa, n):
    """P = R^{-1} xi against the exact (1 - kappa + kappa Delta)^{1/2} xi from a dense
    eigen-decomposition, within the pole set's accuracy (reading of the kappa pole sets), and the
    heat-bath property R(Delta) P = xi to the same order."""
    L = (2, 2, 2, 2)
    U = inputs.random_links(L, "eps", 0.6, seed=81).numpy()
    xi = inputs.gaussian_fields(L, 1, seed=82).numpy()
    c, r, s = ra.kappa_poles(kappa, n)
    P = ra.heatbath_momenta(U, xi, L, kappa, c, r, s)
    D = dense.dense_laplacian(U, L)
    w, Q = dense.eigh(D)
    ysq = Q @ np.diag(np.sqrt(1 - kappa + kappa * w)) @ Q.T
    exact = dense.apply_dense_to_link_field(ysq, xi)
    # relative accuracy of R^2 y on [0, 16]: 2.3e-11 (kappa 0.5, 12 poles), 2.3e-8 (0.9, 16)
    bound = {0.5: 1e-10, 0.9: 1e-7}[kappa]
    assert np.abs(P - exact).max() <= bound * np.abs(exact).max()
    back, _ = ra.rational_apply(U, P, L, c, r, s)
    assert np.abs(back - xi).max() <= bound * np.abs(xi).max()


@pytest.mark.parametrize("kappa,n", [(0.9, 8), (0.5, 4)])
def test_inverse_apply_against_dense(kappa, n):
    """The exact heat bath P = R(Delta)^{-1} xi (CG on R(Delta) P = xi) against the dense
    eigen-decomposition Q diag(1 / R(lambda)) Q^T xi of the adjoint-form matrix, to 1e-10, and for a
    rational with c > 0 (Eq. 6 quadratic terms) as well."""
    L = (2, 2, 2, 2)
    U = inputs.random_links(L, "eps", 0.6, seed=83).numpy()
    xi = inputs.gaussian_fields(L, 1, seed=84).numpy()[0]
    D = dense.dense_laplacian(U, L)
    w, Q = dense.eigh(D)
    for c, r, s in (ra.kappa_poles(kappa, n),
                    ra.poles_from_quadratics(0.4, [0.3, 0.1], [1.0, 0.2], [0.05, 0.3], [0.6, 1.4])):
        P = ra.inverse_apply(U, xi, L, c, r, s, tol=1e-12)
        inv = Q @ np.diag(1.0 / ra.rational_scalar(w, c, r, s)) @ Q.T
        exact = dense.apply_dense_to_link_field(inv, xi)
        assert np.abs(P - exact).max() <= 1e-10 * np.abs(exact).max()
