"""Even-odd (Schur complement) reduction of D(mu).  Test infrastructure: only
tests and benchmarks import this module.

The paper's HMC works with the even-odd reduced operator (Sec. 1.2, where the
comparison solver is even-odd CG).  With the sites split by the parity of
x + y + z + t, the hopping term only connects opposite parities and the
clover plus twisted-mass term is site-diagonal, so

    D = [[D_ee, D_eo], [D_oe, D_oo]],   D_hat = D_ee - D_eo D_oo^-1 D_oe

acts on the even sites, and D x = b is solved by D_hat x_e = b_e - D_eo
D_oo^-1 b_o, x_o = D_oo^-1 (b_o - D_oe x_e).  This is the definition written
out with the oracle's own operator pieces and a per-site dense inverse.
Parity is pinned by the tests against a dense solve of the full system.
"""
from __future__ import annotations

import torch

from .dirac import CDT, WilsonClover


def parity_mask(dims, parity: int) -> torch.Tensor:
    """[T, Z, Y, X] float mask of the sites with (x + y + z + t) % 2 == parity."""
    lx, ly, lz, lt = dims
    t = torch.arange(lt).reshape(lt, 1, 1, 1)
    z = torch.arange(lz).reshape(1, lz, 1, 1)
    y = torch.arange(ly).reshape(1, 1, ly, 1)
    x = torch.arange(lx).reshape(1, 1, 1, lx)
    return (((x + y + z + t) % 2) == parity).to(torch.float64)


class SchurOperator:
    """D_hat(mu) = D_ee - D_eo D_oo^-1 D_oe on fields [..., T, Z, Y, X, 12];
    the odd-site entries of an input are ignored and those of an output are 0."""

    def __init__(self, op: WilsonClover, mu_tm: float):
        self.op = op
        self.mu = float(mu_tm)
        # site-diagonal block: clover (with m0 + 4) plus i mu Gamma5
        self.M = op.A + 1j * self.mu * torch.diag(op.g5).to(CDT)
        self.Minv = torch.linalg.inv(self.M)
        self.even = parity_mask(op.dims, 0)[..., None]
        self.odd = parity_mask(op.dims, 1)[..., None]

    def hop(self, psi):
        out = torch.zeros_like(psi)
        for m in range(4):
            out = out + self.op.hop(psi, m, +1) + self.op.hop(psi, m, -1)
        return out

    def site(self, mat, psi):
        return torch.einsum("...ij,...j->...i", mat, psi)

    def apply(self, psi):
        pe = psi * self.even
        t = self.site(self.Minv, self.hop(pe) * self.odd) * self.odd     # D_oo^-1 D_oe psi_e
        return (self.site(self.M, pe) - self.hop(t)) * self.even

    def reduced_rhs(self, b):
        """b_e - D_eo D_oo^-1 b_o (on the even sites)."""
        t = self.site(self.Minv, b * self.odd) * self.odd
        return (b - self.hop(t)) * self.even

    def odd_solution(self, b, x_e):
        """x_o = D_oo^-1 (b_o - D_oe x_e)."""
        return self.site(self.Minv, (b - self.hop(x_e * self.even)) * self.odd) * self.odd
