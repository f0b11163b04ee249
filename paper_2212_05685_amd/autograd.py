"""Omega as a torch.autograd.Function (App. B: the density matrix is the
derivative of the grand potential; the backward pass is the adjoint Chebyshev
recursion of the library, followed by the builder VJP).

    omega = GrandPotential.apply(n, chi, delta, problem)
    omega = GrandPotentialSDW.apply(n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, problem)

n: float64 [N]; chi, delta: complex128 [4, N] on the GPU (per spin for the
spin-polarised form, whose h is kpm_build_H_sdw and whose backward ends in
kpm_build_H_sdw_vjp).  The spectral
bounds (a, b) and the expansion coefficients are computed in the forward pass
and held constant for differentiation.  Gradients for complex inputs follow
torch's convention dOmega/dRe z + i dOmega/dIm z.
"""
from __future__ import annotations

import torch

from . import kpm
from .solver import KPMProblem


def _adjoint(p: KPMProblem, h, ab, C, gbar):
    """rho from the library's adjoint; when the shared workspace no longer
    holds this forward's checkpoints (another forward ran on the same problem
    in between), the forward recursion is run again first."""
    try:
        return p.grand_potential_grad(h, ab, C, omega_bar=gbar)
    except kpm.KpmError as e:
        if e.status != kpm.KPM_EWORKSPACE:
            raise
    p.grand_potential(h, ab, C)
    return p.grand_potential_grad(h, ab, C, omega_bar=gbar)


class GrandPotential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n, chi, delta, problem: KPMProblem):
        n, chi, delta = n.contiguous(), chi.contiguous(), delta.contiguous()
        h = problem.build_H(n, chi, delta)
        ab = problem.bounds(h)
        C = problem.coefficients(ab)
        omega = problem.grand_potential(h, ab, C)
        ctx.problem = problem
        ctx.save_for_backward(n, chi, delta, h, ab, C)
        return omega.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        n, chi, delta, h, ab, C = ctx.saved_tensors
        p = ctx.problem
        gbar = grad_out.reshape(1).to(torch.float64).contiguous()
        rho = _adjoint(p, h, ab, C, gbar)
        dn, dchi, ddelta = p.build_H_vjp(n, chi, delta, rho)
        return dn, dchi, ddelta, None


class GrandPotentialSDW(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, problem: KPMProblem):
        th = tuple(x.contiguous() for x in (n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn))
        h = problem.build_H_sdw(*th)
        ab = problem.bounds(h)
        C = problem.coefficients(ab)
        omega = problem.grand_potential(h, ab, C)
        ctx.problem = problem
        ctx.save_for_backward(*th, h, ab, C)
        return omega.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        *th, h, ab, C = ctx.saved_tensors
        p = ctx.problem
        gbar = grad_out.reshape(1).to(torch.float64).contiguous()
        rho = _adjoint(p, h, ab, C, gbar)
        return (*p.build_H_sdw_vjp(th, rho), None)
