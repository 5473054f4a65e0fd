"""Non-degenerate twisted-mass doublet operator.  Test infrastructure: only
tests and benchmarks import this module.

Sec. 1.1, Eq. 2: for the heavy (strange-charm) doublet

    D_ND(mubar, epsbar) = D x I_2 + i mubar (Gamma5 x tau_3) - epsbar (I x tau_1)
                        = [[D(mubar), -epsbar], [-epsbar, D(-mubar)]]

with D(+-mubar) the twisted-mass clover operator of the light sector, and
Q_ND = (Gamma5 x tau_1) D_ND its Hermitian form (Sec. 3).  The coarse
doublet operator is the Galerkin product with P_ND = P x I_2 (Sec. 1.1,
after Eq. 2), written out below as prolong, apply, restrict per flavour.  Fields carry the
flavour as their leading axis: [2, T, Z, Y, X, 12].

The unit-link closed form below is the same operator in momentum space: one
8 x 8 matrix (spin x flavour) per momentum, solved by a dense library solve;
it shares no code with the position-space hops and pins them.
"""
from __future__ import annotations

import numpy as np
import torch

from .dirac import CDT, WilsonClover, gammas


class NDOperator:
    """D_ND(mubar, epsbar) on flavour doublets [..., 2, T, Z, Y, X, 12]."""

    def __init__(self, op: WilsonClover, mubar: float, epsbar: float):
        self.op = op
        self.mubar = float(mubar)
        self.epsbar = float(epsbar)

    def apply(self, psi):
        up, dn = psi.unbind(-6)
        out_up = self.op.apply(up, self.mubar) - self.epsbar * dn
        out_dn = self.op.apply(dn, -self.mubar) - self.epsbar * up
        return torch.stack([out_up, out_dn], dim=-6)

    def apply_q(self, psi):
        """Q_ND = (Gamma5 x tau_1) D_ND: swap the flavours, then Gamma5."""
        d = self.apply(psi)
        return self.op.g5 * d.flip(-6)


def free_field_nd_solve(b: torch.Tensor, m0: float, mubar: float, epsbar: float) -> torch.Tensor:
    """x = D_ND^-1 b at U = 1 by FFT (antiperiodic time as in free_field_solve).

    b: [2, T, Z, Y, X, 12].  Per momentum the operator is
    [[S(p) + i mubar g5, -epsbar], [-epsbar, S(p) - i mubar g5]] acting on
    (spin, flavour), S(p) = a(p) + i sum_mu g_mu sin p_mu, a(p) = m0 + sum (1 - cos p).
    """
    lt, lz, ly, lx = b.shape[1:5]
    t = torch.arange(lt, dtype=torch.float64)
    ph = torch.exp(-1j * np.pi * t / lt).to(CDT).reshape(1, lt, 1, 1, 1, 1)
    f = torch.fft.fftn(b * ph, dim=(1, 2, 3, 4))
    g = gammas()
    kt = 2 * np.pi * (torch.arange(lt, dtype=torch.float64) + 0.5) / lt
    kz = 2 * np.pi * torch.arange(lz, dtype=torch.float64) / lz
    ky = 2 * np.pi * torch.arange(ly, dtype=torch.float64) / ly
    kx = 2 * np.pi * torch.arange(lx, dtype=torch.float64) / lx
    PT, PZ, PY, PX = torch.meshgrid(kt, kz, ky, kx, indexing="ij")
    ps = [PX, PY, PZ, PT]
    a = m0 + sum(1.0 - torch.cos(pm) for pm in ps)
    S = a[..., None, None] * torch.eye(4, dtype=CDT)
    for m in range(4):
        S = S + 1j * torch.sin(ps[m])[..., None, None] * g[m]
    e4 = torch.eye(4, dtype=CDT).expand_as(S)
    top = torch.cat([S + 1j * mubar * g[4], -epsbar * e4], dim=-1)
    bot = torch.cat([-epsbar * e4, S - 1j * mubar * g[4]], dim=-1)
    M = torch.cat([top, bot], dim=-2)                                    # [T, Z, Y, X, 8, 8]
    # rhs per momentum: (flavour, spin) rows, colour columns
    ff = f.reshape(2, lt, lz, ly, lx, 4, 3).permute(1, 2, 3, 4, 0, 5, 6).reshape(lt, lz, ly, lx, 8, 3)
    xf = torch.linalg.solve(M, ff)
    xf = xf.reshape(lt, lz, ly, lx, 2, 4, 3).permute(4, 0, 1, 2, 3, 5, 6).reshape(2, lt, lz, ly, lx, 12)
    x = torch.fft.ifftn(xf, dim=(1, 2, 3, 4))
    return x / ph


def coarse_nd_apply(op: WilsonClover, P, mubar: float, epsbar: float, e: torch.Tensor) -> torch.Tensor:
    """D_ND,c e = P_ND^dag D_ND P_ND e with P_ND = P x I_2 (P an oracle
    Prolongation of the light sector): each flavour's coarse field is
    prolonged with P, D_ND acts on the doublet, and each flavour is
    restricted with P^dag.  e: [2, Tc, Zc, Yc, Xc, d]."""
    nd = NDOperator(op, mubar, epsbar)
    w = torch.stack([P.prolong(e[0]), P.prolong(e[1])])
    y = nd.apply(w)
    return torch.stack([P.restrict(y[0]), P.restrict(y[1])])


def sap_doublet(nd: NDOperator, eta: torch.Tensor, blk, sweeps: int, mr_steps: int, block_solver=None) -> torch.Tensor:
    """k sweeps of SAP from zero for D_ND z = eta with the coupled block
    operator: the blocks of one colour (Dirichlet restriction of D_ND, both
    flavours of a block together) are solved by mr_steps of minimal
    residual, one alpha per block from sums over both flavours' sites.
    eta: [2, T, Z, Y, X, 12].  block_solver(r, mask) -> e replaces the MR
    steps (the exact solves of the pins)."""
    from .mg import block_colour, check_blocking, to_blocks
    op = nd.op
    check_blocking(op.dims, blk)
    colour = block_colour(op.dims, blk)
    bx, by, bz, bt = blk

    def bsum(f):   # per-block sums over sites and both flavours
        return to_blocks(f, blk, False).sum(-1).sum(0)

    def expand(a):
        a = a.repeat_interleave(bt, dim=-4).repeat_interleave(bz, dim=-3)
        return a.repeat_interleave(by, dim=-2).repeat_interleave(bx, dim=-1)[..., None]

    z = torch.zeros_like(eta)
    for _ in range(sweeps):
        for c in (0, 1):
            mask = (colour == c).to(torch.float64)[..., None]
            r = mask * (eta - nd.apply(z))
            if block_solver is not None:
                z = z + block_solver(r, mask)
                continue
            e = torch.zeros_like(r)
            rho = r.clone()
            for _ in range(mr_steps):
                q = mask * nd.apply(mask * rho)
                qq = bsum((q.conj() * q).real)
                qr = bsum(q.conj() * rho)
                alpha = torch.where(qq > 0, qr / torch.where(qq > 0, qq, torch.ones_like(qq)),
                                    torch.zeros_like(qr))
                a = expand(alpha)
                e = e + a * rho
                rho = rho - a * q
            z = z + e
    return z
