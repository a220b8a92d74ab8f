"""Pins for oracle.leapfrog, the implicit leapfrog step of the non-separable RMHMC Hamiltonian
(CPU): the reduction to the explicit leapfrog for a constant mass term, time reversibility,
the third-order local energy error and SU(3) links."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import gauge, leapfrog, rational, su3
from paper_2112_04556_amd import inputs

L = (2, 2, 2, 4)
BETA = 5.0


def _state(seed=3):
    U = inputs.random_links(L, "eps", 0.5, seed=seed).numpy()
    P = inputs.gaussian_fields(L, 1, seed=seed).numpy()[0]
    return U, P


def _poles():
    c, r, s = rational.kappa_poles(0.5, 4)
    return c, np.asarray(r), np.asarray(s)


def test_constant_mass_is_the_explicit_leapfrog():
    """R = 1 (c = 1, a pole of weight 0): Pi = P and the kinetic force vanishes, so the step is the
    textbook leapfrog P_h = P + h F_G(U), U' = exp(i eps P_h) U, P' = P_h + h F_G(U')."""
    U, P = _state()
    eps = 0.2
    U1, P1, ip, iu = leapfrog.glf_step(U, P, L, 1.0, np.array([0.0]), np.array([1.0]), BETA, eps)
    h = eps / 2
    Ph = P + h * gauge.gauge_force(U, L, BETA)
    H = np.einsum("mav,aij->mvij", Ph.astype(np.complex128), su3.T)
    Ue = expm(1j * eps * H) @ U
    Pe = Ph + h * gauge.gauge_force(Ue, L, BETA)
    assert np.abs(U1 - Ue).max() <= 1e-13
    assert np.abs(P1 - Pe).max() <= 1e-12
    assert ip <= 2 and iu <= 2


def test_reversible():
    """The step from (U', -P') returns to (U, -P) within the fixed-point tolerance."""
    U, P = _state()
    c, r, s = _poles()
    U1, P1, ip, iu = leapfrog.glf_step(U, P, L, c, r, s, BETA, 0.1)
    assert ip > 2 and iu > 2            # the fixed points are really iterated
    U2, P2, _, _ = leapfrog.glf_step(U1, -P1, L, c, r, s, BETA, 0.1)
    assert np.abs(U2 - U).max() <= 1e-10
    assert np.abs(P2 + P).max() <= 1e-10 * np.abs(P).max()
    assert np.abs(U1 - U).max() > 1e-3  # the links did move


def test_energy_error_is_third_order():
    """A symmetric second-order step changes H by O(eps^3) (here with a large eps^4 term as well:
    dH ~ -0.8 eps^3 - 35 eps^4 on this state): halving eps divides |dH| by 8 to 16, where a
    first-order mistake (a wrong sign or factor in a force, an unsymmetric stage) gives 2 to 4."""
    U, P = _state(seed=5)
    c, r, s = _poles()
    H0 = leapfrog.hamiltonian(U, P, L, c, r, s, BETA)
    dH = []
    for eps in (0.05, 0.025):
        U1, P1, _, _ = leapfrog.glf_step(U, P, L, c, r, s, BETA, eps)
        dH.append(leapfrog.hamiltonian(U1, P1, L, c, r, s, BETA) - H0)
    ratio = abs(dH[0]) / abs(dH[1])
    assert 7.0 < ratio < 17.0, (dH, ratio)
    assert abs(dH[0]) < 1e-4 * abs(H0)


def test_links_stay_in_su3():
    U, P = _state(seed=7)
    c, r, s = _poles()
    U1, _, _, _ = leapfrog.glf_step(U, P, L, c, r, s, BETA, 0.3)
    eye = np.eye(3)
    assert np.abs(U1 @ np.conj(np.swapaxes(U1, -1, -2)) - eye).max() <= 1e-13
    assert np.abs(np.linalg.det(U1) - 1.0).max() <= 1e-13


def test_velocity_is_r_squared():
    """Pi = R(Delta)^2 P: on U = 1 every plane wave is an eigenvector of Delta, so Pi of a single
    mode is R(lambda)^2 times it (lambda = sum_mu 2 - 2 cos k_mu on the free lattice)."""
    Lf = (4, 2, 2, 2)
    U = inputs.random_links(Lf, "unit").numpy()
    V = int(np.prod(Lf))
    x0 = np.arange(V) % Lf[0]
    mode = np.cos(2 * np.pi * x0 / Lf[0])        # k = (2 pi / 4, 0, 0, 0): lambda = 2
    P = np.zeros((4, 8, V))
    P[1, 3] = mode
    c, r, s = _poles()
    pi = leapfrog.velocity(U, P, Lf, c, r, s)
    R = rational.rational_scalar(2.0, c, r, s)
    assert np.abs(pi - R * R * P).max() <= 1e-11
