"""Oracle: the pseudofermion action S_f = phi^dag (D D^dag)^-1 phi and its force.

The paper computes the force terms of its monomials with DD-alpha-AMG
(Sec. 1.2, stopping criterion 1e-9 for forces); the force itself is the
standard one.  With Y = D^-1 phi and X = (D^dag)^-1 Y = (D D^dag)^-1 phi,
    dS_f = -2 Re < X, dD Y >.
The oracle does not derive dD by hand: it differentiates the surrogate
    L(U) = -2 Re < X0, D[U] Y0 >     (X0, Y0 held fixed)
with torch autograd through the hopping term and the clover leaves, whose
gradient at U equals that of S_f.

Tangent convention: U_mu(x) -> exp(t w) U_mu(x), w in su(3), generators
T^a = i lambda^a / 2 (tr T^a T^b = -delta_ab / 2).  The force is
F_mu(x) = sum_a (dS/dw^a) T^a, so dS/dt = -2 sum tr(F w).  If
dS/dt = Re tr(M w) for all w then F = -1/2 TA(M) with
TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6.  For torch's gradient g of a real
function (dS = Re tr(g^dag dU)) and dU = w U, M = U g^dag.
"""
from __future__ import annotations

import torch

from .dirac import CDT, WilsonClover, dag


def traceless_antihermitian(m: torch.Tensor) -> torch.Tensor:
    a = 0.5 * (m - dag(m))
    tr = torch.diagonal(a, dim1=-2, dim2=-1).sum(-1)
    return a - (tr / 3.0)[..., None, None] * torch.eye(3, dtype=CDT)


def force_from_fields(U, m0: float, csw: float, X: torch.Tensor, Y: torch.Tensor,
                      antiperiodic: bool = True) -> torch.Tensor:
    """F_mu(x) for fixed X, Y: [4, T, Z, Y, X, 3, 3] traceless anti-Hermitian."""
    Ut = torch.as_tensor(U, dtype=CDT).detach().clone().requires_grad_(True)
    op = WilsonClover(Ut, m0, csw, antiperiodic)
    DY = op.apply(Y.detach(), 0.0)
    L = -2.0 * torch.sum(X.detach().conj() * DY).real
    (g,) = torch.autograd.grad(L, Ut)
    M = Ut.detach() @ dag(g)
    return -0.5 * traceless_antihermitian(M)


def action_and_force(U, m0: float, csw: float, mu_tm: float, phi: torch.Tensor, solve):
    """S_f and F with a caller-supplied solver solve(b, mu) ~ D(mu)^-1 b.

    Y = D(mu)^-1 phi; X = (D(mu)^dag)^-1 Y = Gamma5 D(-mu)^-1 Gamma5 Y.
    """
    op = WilsonClover(U, m0, csw)
    Y = solve(phi, mu_tm)
    X = op.g5 * solve(op.g5 * Y, -mu_tm)
    S = float(torch.sum(phi.conj() * X).real)
    return S, force_from_fields(U, m0, csw, X, Y), X, Y


def directional_derivative(F: torch.Tensor, omega: torch.Tensor) -> float:
    """dS/dt along U -> exp(t omega) U: -2 sum tr(F omega)."""
    return float(-2.0 * torch.einsum("...ij,...ji->", F, omega).real)
