"""Rational mass term, shifted solves and the kinetic energy (oracle; test infrastructure only).

Section 3, Eq. 6 writes the mass term as M = [c + sum_i (a0_i + a1_i L)/(b0_i + b1_i L + L^2)]^(-2)
with L = -nabla^2_G/16 = Delta/16, and Eq. 5 puts 1/2 P M^{-1} P in the
Hamiltonian.  With R(Delta) = c + sum_i (...), M^{-1} = R^2, so the kinetic energy
is K = 1/2 <Y, Y> with Y = R(Delta) P.  Readings (listed in the design doc):

* each quadratic term with real distinct roots splits into two real poles
  rho/(L + s); in Delta units a pole is r/(Delta + sigma) with r = 16 rho,
  sigma = 16 s.  Complex or repeated roots are rejected;
* K = 1/2 sum over components (so the M = 1 heatbath draws P^a ~ N(0, 1));
* the "(1 - kappa + kappa Delta)^-1-type" pole sets: R ~ y^(-1/2) with
  y = 1 - kappa + kappa Delta, by the midpoint rule on
  y^(-1/2) = (2/pi) sqrt(s) int_0^{pi/2} dtheta / (s sin^2 theta + y cos^2 theta),
  s = sqrt((1 - kappa)(1 + 15 kappa)).

The shifted systems (Delta + sigma_j) x_j = b are solved one shift at a time by
plain conjugate gradients from a zero guess; that is the definition of
(Delta + sigma_j)^{-1} b up to the stated tolerance.
"""
from __future__ import annotations

import numpy as np

from .laplacian import inner, laplacian


def poles_from_quadratics(c, a0, a1, b0, b1):
    """Eq. 6 terms (in L = Delta/16 units) -> (c, r[], sigma[]) in Delta units."""
    r, sigma = [], []
    for A0, A1, B0, B1 in zip(a0, a1, b0, b1):
        disc = B1 * B1 - 4.0 * B0
        if not disc > 0.0:
            raise ValueError("quadratic term without two distinct real roots")
        sq = np.sqrt(disc)
        s1, s2 = (B1 - sq) / 2.0, (B1 + sq) / 2.0   # L^2 + B1 L + B0 = (L + s1)(L + s2)
        rho1 = (A0 - A1 * s1) / (s2 - s1)
        rho2 = (A0 - A1 * s2) / (s1 - s2)
        for rho, s in ((rho1, s1), (rho2, s2)):
            if not s > 0.0:
                raise ValueError("pole with non-positive shift")
            r.append(16.0 * rho)
            sigma.append(16.0 * s)
    return float(c), np.array(r), np.array(sigma)


def quadratic_term(lam, a0, a1, b0, b1):
    """(a0 + a1 L)/(b0 + b1 L + L^2) at L = lambda/16, evaluated directly."""
    Lv = np.asarray(lam, np.float64) / 16.0
    return (a0 + a1 * Lv) / (b0 + b1 * Lv + Lv * Lv)


def kappa_poles(kappa: float, n: int):
    """(c, r[], sigma[]) with R(Delta)^2 ~ (1 - kappa + kappa Delta)^-1 on Delta in [0, 16].

    Midpoint rule with nodes theta_j = (2j - 1) pi/(4n), j = 1..n:
    r_j = sqrt(s)/(n kappa cos^2 theta_j), sigma_j = (1 - kappa + s tan^2 theta_j)/kappa.
    """
    s = np.sqrt((1.0 - kappa) * (1.0 + 15.0 * kappa))
    th = (2.0 * np.arange(1, n + 1) - 1.0) * np.pi / (4.0 * n)
    r = np.sqrt(s) / (n * kappa * np.cos(th) ** 2)
    sigma = (1.0 - kappa + s * np.tan(th) ** 2) / kappa
    return 0.0, r, sigma


def rational_scalar(lam, c, r, sigma):
    """R(lambda) = c + sum_j r_j/(lambda + sigma_j) on numbers."""
    lam = np.asarray(lam, np.float64)
    return c + sum(rj / (lam + sj) for rj, sj in zip(r, sigma))


def cg_solve(U, b, L, sigma: float, tol: float = 1e-13, maxiter: int = 100000):
    """Plain CG for (Delta + sigma) x = b from x = 0, one field b of shape (4, 8, V).

    Stops when the recomputed residual ||b - (Delta + sigma) x|| <= tol ||b||.
    Returns (x, iterations, final relative residual).
    """
    b = np.asarray(b, np.float64)
    bnorm = np.sqrt(inner(b, b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    p = r.copy()
    rr = inner(r, r)
    it = 0
    while it < maxiter:
        Ap = laplacian(U, p, L, sigma)
        alpha = rr / inner(p, Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = inner(r, r)
        it += 1
        if np.sqrt(rr_new) <= tol * bnorm:
            true_r = b - laplacian(U, x, L, sigma)
            res = np.sqrt(inner(true_r, true_r)) / bnorm
            if res <= tol:
                return x, it, res
            r = true_r            # restart from the true residual
            rr_new = inner(r, r)
            p = r.copy()
            rr = rr_new
            continue
        p = r + (rr_new / rr) * p
        rr = rr_new
    true_r = b - laplacian(U, x, L, sigma)
    return x, it, np.sqrt(inner(true_r, true_r)) / bnorm


def shifted_solves(U, b, L, sigma, tol: float = 1e-13):
    """x[j] = (Delta + sigma_j)^{-1} b for a field b of shape (4, 8, V)."""
    return np.stack([cg_solve(U, b, L, s, tol)[0] for s in sigma])


def rational_apply(U, x, L, c, r, sigma, tol: float = 1e-13):
    """(y, x_poles): y = c x + sum_j r_j (Delta + sigma_j)^{-1} x, x of shape (n, 4, 8, V)."""
    x = np.asarray(x, np.float64)
    ys, xps = [], []
    for xi in x:
        xp = shifted_solves(U, xi, L, sigma, tol)
        ys.append(c * xi + np.tensordot(np.asarray(r), xp, axes=1))
        xps.append(xp)
    return np.stack(ys), np.stack(xps)


def kinetic_energy(U, P, L, c, r, sigma, tol: float = 1e-13):
    """K[n] = 1/2 <Y_n, Y_n> with Y = R(Delta) P (Eq. 5 with M^{-1} = R^2, Eq. 6)."""
    Y, _ = rational_apply(U, P, L, c, r, sigma, tol)
    return 0.5 * np.sum((Y * Y).reshape(Y.shape[0], -1), axis=1), Y


def heatbath_momenta(U, xi, L, kappa: float, c, r, sigma, tol: float = 1e-13):
    """Heat-bath momenta for the kinetic term 1/2 P M^{-1} P with M = R^{-2} (section 3):
    P = M^{1/2} xi = R(Delta)^{-1} xi.  For the pole sets with R^2 ~ y^{-1}, y = 1 - kappa + kappa
    Delta, R^{-1} ~ y^{1/2} = y R, so P = (1 - kappa) R xi + kappa Delta (R xi)."""
    y, _ = rational_apply(U, xi, L, c, r, sigma, tol)
    return (1.0 - kappa) * y + kappa * laplacian(U, y, L)


def inverse_apply(U, x, L, c, r, sigma, tol: float = 1e-12, maxiter: int = 1000, inner_tol: float = 1e-14):
    """P = R(Delta)^{-1} x for one field x of shape (4, 8, V), by plain CG on R(Delta) P = x, each
    application of R(Delta) being rational_apply (R(lambda) > 0 on the spectrum [0, 16] makes R(Delta)
    symmetric positive definite).  The heat bath of section 3 with M = R^{-2} is P = R(Delta)^{-1} xi.
    Stops when the residual ||x - R(Delta) P|| <= tol ||x||; the inner shifted solves run to
    inner_tol."""
    x = np.asarray(x, np.float64)
    bnorm = np.sqrt(inner(x, x))
    P = np.zeros_like(x)
    if bnorm == 0.0:
        return P
    res = x.copy()
    p = res.copy()
    rr = inner(res, res)
    for _ in range(maxiter):
        Ap = rational_apply(U, p[None], L, c, r, sigma, inner_tol)[0][0]
        alpha = rr / inner(p, Ap)
        P += alpha * p
        res -= alpha * Ap
        rr_new = inner(res, res)
        if np.sqrt(rr_new) <= tol * bnorm:
            return P
        p = res + (rr_new / rr) * p
        rr = rr_new
    raise RuntimeError("inverse_apply did not converge")
