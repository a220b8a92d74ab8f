"""torch.autograd wrappers of the RMHMC kinetic energy (section 3, Eq. 5 with Eq. 6) and of the
Chebyshev power spectrum (section 2, Eq. 4).

K(omega, P) = 1/2 sum_n <Y_n, Y_n>,  Y = R(Delta[exp(i omega.T) U]) P.  ``omega`` is the
(4, 8, V) Lie-algebra displacement of every link under left multiplication (the derivative
convention of section 2).  At omega = 0 its gradient is the kinetic (mass-term) force with the
opposite sign, F_M = -dK/d omega; at omega != 0 the forward displaces the links
(rmh_link_exp) and the backward carries the derivative at the displaced links through the
differential of the exponential map (rmh_link_exp_vjp), so torch.autograd.gradcheck sees a real
function of omega.  The backward recomputes both multi-shift solves in the HIP library (no
solution is stored).
"""
from __future__ import annotations

import torch

from . import api


class KineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega, P, U, L, rat, solver):
        if omega.shape != (4, 8, api.volume(L)):
            raise ValueError("omega must have shape (4, 8, V)")
        displaced = bool(torch.any(omega != 0))
        Uw = api.link_exp(L, U, omega.contiguous()) if displaced else U
        out = api.rational_apply(L, Uw, P, rat, solver, want_K=True)
        ctx.save_for_backward(P, out["y"], Uw, omega)
        ctx.L, ctx.rat, ctx.solver, ctx.displaced = L, rat, solver, displaced
        return torch.tensor(float(out["K"].sum()), dtype=torch.float64, device=P.device)

    @staticmethod
    def backward(ctx, gK):
        P, Y, Uw, omega = ctx.saved_tensors
        gx, go, _ = api.rational_apply_bwd(ctx.L, Uw, P, Y, ctx.rat, ctx.solver,
                                           grad_x=ctx.needs_input_grad[1], per_rhs=False)
        grad_omega = None
        if ctx.needs_input_grad[0]:
            g = go[0]
            if ctx.displaced:
                g = api.link_exp_vjp(ctx.L, omega.contiguous(), g)
            grad_omega = g * gK
        grad_P = gx * gK if gx is not None else None
        return grad_omega, grad_P, None, None, None, None


def kinetic_energy(omega, P, U, L, rat, solver=api.Solver()):
    return KineticEnergy.apply(omega, P, U, L, rat, solver)


class PowerSpectrum(torch.autograd.Function):
    """power[n, w] = <F_n, B_w(Delta[exp(i omega.T) U]) F_n> (FP64), omega displacing the links as in
    KineticEnergy.  The backward runs the reverse Chebyshev sweep in the HIP library: gradients for
    omega and F."""

    @staticmethod
    def forward(ctx, omega, F, U, L, degree, n_windows, edges, kernel):
        if omega.shape != (4, 8, api.volume(L)):
            raise ValueError("omega must have shape (4, 8, V)")
        displaced = bool(torch.any(omega != 0))
        Uw = api.link_exp(L, U, omega.contiguous()) if displaced else U
        _, pw = api.power_spectrum(L, Uw, F, degree, n_windows, edges, kernel)
        ctx.save_for_backward(F, Uw, omega)
        ctx.args = (L, degree, n_windows, edges, kernel)
        ctx.displaced = displaced
        return torch.from_numpy(pw).to(F.device)

    @staticmethod
    def backward(ctx, gp):
        F, Uw, omega = ctx.saved_tensors
        L, degree, n_windows, edges, kernel = ctx.args
        gF, go = api.power_spectrum_bwd(L, Uw, F, gp.detach().cpu().double().numpy(), degree, n_windows, edges,
                                        kernel, grad_F=ctx.needs_input_grad[1],
                                        grad_omega=ctx.needs_input_grad[0])
        g = None
        if go is not None:
            g = go[0]
            if ctx.displaced:
                g = api.link_exp_vjp(L, omega.contiguous(), g)
        return g, gF, None, None, None, None, None, None


def power_spectrum(omega, F, U, L, degree, n_windows, edges=None, kernel=1):
    return PowerSpectrum.apply(omega, F, U, L, degree, n_windows, edges, kernel)
