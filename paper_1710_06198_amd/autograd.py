"""The pseudofermion action as a differentiable PyTorch function.

S_f = phi^dag (D D^dag)^-1 phi (the action whose force Sec. 1.2 of the paper
computes with DD-alpha-AMG) is evaluated by the library (two multigrid
solves) and differentiated by its adjoint kernels (the force), both through
the C ABI; this module only connects them to autograd.

The links live on SU(3), so the gradient is the one on the group: for every
perturbation U -> exp(X) U with X traceless anti-Hermitian, the first-order
change of S_f is Re sum conj(U.grad) (X U), i.e. U.grad is PyTorch's complex
gradient (dS/dRe U + i dS/dIm U) on the directions tangent to SU(3).  Its
component normal to the group is not computed, so it is meant for updates
that stay on the group (HMC momenta, exp(-eps F) U), not for gradient steps
on unconstrained complex matrices.
"""
from __future__ import annotations

import torch


class FermionAction(torch.autograd.Function):
    """S = FermionAction.apply(U, phi, solver, kappa, csw, mu, tol, update_iters).

    U: links, complex128 [4][T][Z][Y][X][3][3] on the solver's device.
    phi: pseudofermion, complex128 [1][T][Z][Y][X][4][3].
    solver: a paper_1710_06198_amd.Solver for the lattice; the first call
    runs its full setup at (kappa, csw, mu), later calls move it to the new
    links with `update_iters` setup iterations (the paper's setup update).
    Returns S_f as a 0-dim float64 tensor; backward gives U.grad (see the
    module docstring) and no gradient for phi.
    """

    @staticmethod
    def forward(ctx, U, phi, solver, kappa, csw, mu, tol=1e-12, update_iters=1):
        U = U.contiguous()
        if getattr(solver, "_action_setup", None) == (float(kappa), float(csw), float(mu)):
            solver.setup_update(U, update_iters)
        else:
            solver.setup(U, kappa, csw, mu)
            solver._action_setup = (float(kappa), float(csw), float(mu))
        F = torch.empty_like(U)
        S, info = solver.force(phi.contiguous(), F, tol=tol)
        if info.status != 0:
            raise RuntimeError(f"pseudofermion solves did not converge: {info.as_dict()}")
        ctx.solver = solver
        ctx.version = solver.links_version
        ctx.save_for_backward(F)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, grad_S):
        (F,) = ctx.saved_tensors
        if ctx.solver.links_version != ctx.version:
            raise RuntimeError("the solver's links changed between the action and its gradient")
        G = torch.empty_like(F)
        ctx.solver.force_link_gradient(F, G, float(grad_S))
        return G, None, None, None, None, None, None, None


def fermion_action(U, phi, solver, kappa, csw, mu, tol=1e-12, update_iters=1):
    return FermionAction.apply(U, phi, solver, kappa, csw, mu, tol, update_iters)
