"""Oracle: the Wilson plaquette gauge action and its force.  Test
infrastructure: only tests and benchmarks import this module.

The paper's HMC (Sec. 2) places the gauge action on the innermost time
scale of its integrator; its form is the standard one:

    S_g(U) = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3),
    P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,

with periodic links in every direction (the antiperiodic sign belongs to
the fermion field).  The force uses the fermion force's convention
(U -> exp(t w) U, T^a = i lambda^a/2, F = sum_a (dS/dw^a) T^a, so
dS/dt = -2 sum tr(F w)) and is obtained by torch autograd of S_g, projected
as F = -1/2 TA(U g^dag).
"""
from __future__ import annotations

import torch

from .dirac import CDT, dag
from .force import traceless_antihermitian


def _shift(U, mu, step):
    """U(x + step mu), periodic; U: [..., T, Z, Y, X, 3, 3]."""
    return torch.roll(U, shifts=-step, dims=-3 - mu)


def plaquettes(U) -> torch.Tensor:
    """Re tr P_{mu nu}(x) for the six planes mu < nu: [6, T, Z, Y, X]."""
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = U[mu] @ _shift(U[nu], mu, 1) @ dag(_shift(U[mu], nu, 1)) @ dag(U[nu])
            out.append(torch.diagonal(P, dim1=-2, dim2=-1).sum(-1).real)
    return torch.stack(out)


def action(U, beta: float) -> torch.Tensor:
    return beta * torch.sum(1.0 - plaquettes(U) / 3.0)


def force(U, beta: float) -> torch.Tensor:
    """F_mu(x) = sum_a (dS_g/dw^a) T^a: [4, T, Z, Y, X, 3, 3]."""
    Ut = torch.as_tensor(U, dtype=CDT).detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(action(Ut, beta), Ut)
    return -0.5 * traceless_antihermitian(Ut.detach() @ dag(g))
