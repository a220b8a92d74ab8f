"""Implicit (generalized) leapfrog step of RMHMC (oracle; test infrastructure only).

Section 3 notes that the mass term makes the Hamiltonian non-separable, so the molecular-dynamics
step has to be the implicit leapfrog of Girolami and Calderhead (2011).  The Hamiltonian built
here is the kinetic term plus the gauge action,

    H(U, P) = K(U, P) + S_W(U),   K = 1/2 <Y, Y>,  Y = R(Delta[U]) P   (Eq. 5 with M^-1 = R^2),

without the log|M| term: the paper realises that term through auxiliary fields it does not
define.  Links move by left multiplication, U -> exp(i omega^a T^a) U, as in the force of
section 3, so the equations of motion are

    dU/dt = i Pi^a T^a U,   Pi = dH/dP = R(Delta)^2 P,
    dP/dt = F = -dH/d omega = F_G - dK/d omega.

One step of size eps, h = eps / 2, in three stages:

    (i)   P_h = P + h F(U, P_h)                             fixed point in P_h
    (ii)  U'  = exp(i h [Pi(U, P_h) + Pi(U', P_h)]^a T^a) U   fixed point in U'
    (iii) P'  = P_h + h F(U', P_h)                           explicit

Each fixed point x = G(x) is iterated from the explicit guess, x_{k+1} = G(x_k), until successive
iterates differ by at most fp_tol relative to the new one, and the new iterate x_{k+1} is kept
(stage ii iterates Pi(U', P_h) and rebuilds U' from the new Pi).  Any other stopping rule within
fp_tol (for instance keeping x_k) differs from this one by at most fp_tol relative in the fixed
point.  Pi is linear in P, so the step run from (U', -P') returns to (U, -P): the scheme is time
reversible.

Everything is written from the definitions with the oracle's own rational solves, kinetic-force
derivative, gauge force and scipy's matrix exponential.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import gauge, su3
from .force import kinetic_force_grad
from .rational import kinetic_energy, rational_apply


def hamiltonian(U, P, L, c, r, sigma, beta: float, tol: float = 1e-13) -> float:
    """H = 1/2 <R(Delta) P, R(Delta) P> + S_W(U) for one momentum field P of shape (4, 8, V)."""
    K, _ = kinetic_energy(U, np.asarray(P)[None], L, c, r, sigma, tol)
    return float(K[0]) + float(gauge.wilson_action(U, L, beta))


def velocity(U, P, L, c, r, sigma, tol: float = 1e-13) -> np.ndarray:
    """Pi = dH/dP = R(Delta)^2 P, shape (4, 8, V)."""
    y, _ = rational_apply(U, np.asarray(P)[None], L, c, r, sigma, tol)
    z, _ = rational_apply(U, y, L, c, r, sigma, tol)
    return z[0]


def total_force(U, P, L, c, r, sigma, beta: float, tol: float = 1e-13) -> np.ndarray:
    """F = -dH/d omega = F_G(U) - dK/d omega (U, P), shape (4, 8, V)."""
    return gauge.gauge_force(U, L, beta) - kinetic_force_grad(U, np.asarray(P)[None], L, c, r, sigma, tol)


def link_update(U, A) -> np.ndarray:
    """exp(i A^a T^a) U_mu(x) for every link; U (4, V, 3, 3), A (4, 8, V)."""
    H = su3.to_matrix(np.moveaxis(np.asarray(A, np.float64), 1, -1))   # (4, V, 3, 3) Hermitian
    return expm(1j * H) @ np.asarray(U)


def glf_step(U0, P0, L, c, r, sigma, beta: float, eps: float, fp_tol: float = 1e-12, fp_maxiter: int = 50,
             tol: float = 1e-13):
    """(U', P', iterations of stage i, iterations of stage ii) for one step of size eps."""
    U0 = np.asarray(U0)
    P0 = np.asarray(P0, np.float64)
    h = 0.5 * eps
    # (i) P_h = P0 + h F(U0, P_h)
    fg = gauge.gauge_force(U0, L, beta)
    Ph = P0.copy()
    it_p = 0
    while True:
        it_p += 1
        Pn = P0 + h * (fg - kinetic_force_grad(U0, Ph[None], L, c, r, sigma, tol))
        d = np.linalg.norm(Pn - Ph)
        Ph = Pn
        if d <= fp_tol * np.linalg.norm(Pn):
            break
        if it_p >= fp_maxiter:
            raise RuntimeError("stage i did not converge")
    # (ii) U1 = exp(i h (Pi(U0, P_h) + Pi(U1, P_h))) U0, from the guess Pi(U1) = Pi(U0)
    pi0 = velocity(U0, Ph, L, c, r, sigma, tol)
    pi = pi0
    U1 = link_update(U0, h * (pi0 + pi))
    it_u = 0
    while True:
        it_u += 1
        pn = velocity(U1, Ph, L, c, r, sigma, tol)
        d = np.linalg.norm(pn - pi)
        pi = pn
        U1 = link_update(U0, h * (pi0 + pi))
        if d <= fp_tol * np.linalg.norm(pn):
            break
        if it_u >= fp_maxiter:
            raise RuntimeError("stage ii did not converge")
    # (iii) P1 = P_h + h F(U1, P_h)
    P1 = Ph + h * total_force(U1, Ph, L, c, r, sigma, beta, tol)
    return U1, P1, it_p, it_u
