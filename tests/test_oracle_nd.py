"""Pins of the oracle's non-degenerate doublet operator (Sec. 1.1, Eq. 2)
against what the mathematics fixes: the unit-link momentum-space form (an
8 x 8 spin-flavour matrix per momentum, solved by FFT), the Hermiticity of
Q_ND = (Gamma5 x tau_1) D_ND on random SU(3) links (Sec. 3), the
decoupled case epsbar = 0, which reduces to two light-sector closed forms,
and the coarse doublet operator against its Galerkin definition."""
import numpy as np
import pytest
import torch

from lattice_inputs import gauge_links, gaussian_spinor, unit_links
from oracle.dirac import WilsonClover, free_field_solve, spinor_to_field, vdot, norm
from oracle.nd import NDOperator, free_field_nd_solve, coarse_nd_apply, sap_doublet


def doublet(dims, seed):
    return spinor_to_field(gaussian_spinor(dims, seed, n=2))


@pytest.mark.parametrize("mubar,epsbar", [(0.13, 0.11), (0.05, 0.2), (0.0, 0.3)])
def test_unit_link_nd_matches_momentum_space_solve(mubar, epsbar):
    dims = (4, 4, 4, 6)
    m0 = -0.2
    op = WilsonClover(unit_links(dims), m0, 1.7)   # the clover term vanishes at U = 1
    nd = NDOperator(op, mubar, epsbar)
    b = doublet(dims, 41)
    x = free_field_nd_solve(b, m0, mubar, epsbar)
    assert norm(nd.apply(x) - b) / norm(b) < 1e-12


def test_decoupled_doublet_is_two_light_solves():
    dims = (4, 4, 2, 6)
    m0, mu = -0.25, 0.09
    b = doublet(dims, 7)
    x = free_field_nd_solve(b, m0, mu, 0.0)
    assert norm(x[0] - free_field_solve(b[0], m0, mu)) / norm(x[0]) < 1e-12
    assert norm(x[1] - free_field_solve(b[1], m0, -mu)) / norm(x[1]) < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_q_nd_is_hermitian(seed):
    dims = (4, 4, 4, 4)
    op = WilsonClover(gauge_links(dims, seed=seed, eps=0.4), -0.1, 1.6)
    nd = NDOperator(op, 0.12, 0.15)
    a, c = doublet(dims, 10 + seed), doublet(dims, 20 + seed)
    lhs = vdot(a, nd.apply_q(c))
    rhs = vdot(nd.apply_q(a), c)
    assert abs(lhs - rhs) < 1e-11 * norm(a) * norm(c)
    # the same flavour swap with +mubar in both flavours is not Hermitian:
    # the sign of the twist in the second flavour is what Eq. 2 fixes
    q_bad = lambda f: op.g5 * torch.stack([op.apply(f[1], 0.12) - 0.15 * f[0],
                                           op.apply(f[0], 0.12) - 0.15 * f[1]])
    assert abs(vdot(a, q_bad(c)) - vdot(q_bad(a), c)) > 1e-3 * norm(a) * norm(c)


def test_coarse_doublet_operator_is_coupled_light_coarse_operators():
    """D_ND,c = P_ND^dag D_ND P_ND (P_ND = P x I_2) equals each flavour's
    Galerkin D_c(+-mubar) coupled by -epsbar times the identity, because
    P^dag P = I: the flavour coupling survives the coarsening unchanged.
    Checked with an orthonormal P from random test vectors, with epsbar
    above and below mubar."""
    from oracle import mg
    dims = (4, 4, 4, 4)
    op = WilsonClover(gauge_links(dims, 0.35, 71), -0.25, 1.3)
    V = torch.as_tensor(gaussian_spinor(dims, 72, n=5, dof=(12,)))
    P = mg.build_prolongation(V, (2, 2, 2, 2), dims, 12)
    Dc = mg.galerkin(op, P)
    e = torch.as_tensor(gaussian_spinor(P.coarse_dims, 73, n=2, dof=(2 * P.nv,)))
    for mubar, epsbar in ((0.12, 0.10), (0.05, 0.12)):
        got = coarse_nd_apply(op, P, mubar, epsbar, e)
        want = torch.stack([Dc.apply(e[0], mubar) - epsbar * e[1], Dc.apply(e[1], -mubar) - epsbar * e[0]])
        assert norm(got - want) < 1e-13 * norm(want)


def _nd_dense(nd, dims):
    n = 2 * int(np.prod(dims)) * 12
    lx, ly, lz, lt = dims
    eye = torch.eye(n, dtype=torch.complex128).reshape(n, 2, lt, lz, ly, lx, 12)
    return nd.apply(eye).reshape(n, n).T.contiguous()


def test_doublet_sap_exact_blocks():
    """The doublet's SAP with exact solves of the coupled block systems: the
    residual on the just-smoothed colour's blocks vanishes, and one block
    covering the lattice gives D_ND^-1."""
    dims = (4, 4, 2, 2)
    op = WilsonClover(gauge_links(dims, 0.35, 91), -0.3, 1.2)
    nd = NDOperator(op, 0.05, 0.12)
    M = _nd_dense(nd, dims)
    eta = doublet(dims, 92)

    def exact(r, mask):
        m = mask.expand_as(r).reshape(-1).bool()
        idx = torch.nonzero(m).squeeze(1)
        e = torch.zeros(r.numel(), dtype=torch.complex128)
        e[idx] = torch.linalg.solve(M[idx][:, idx], r.reshape(-1)[idx])
        return e.reshape(r.shape)

    from oracle.mg import block_colour
    blk = (2, 2, 2, 2)
    z = sap_doublet(nd, eta, blk, 1, 0, block_solver=exact)
    mask1 = (block_colour(dims, blk) == 1).to(torch.float64)[..., None]
    assert norm(mask1 * (eta - nd.apply(z))) < 1e-12 * norm(eta)
    z = sap_doublet(nd, eta, dims, 1, 0, block_solver=exact)
    assert norm(nd.apply(z) - eta) < 1e-12 * norm(eta)


def test_doublet_sap_mr_reduces_the_residual():
    """More MR steps per coupled block solve never raise the residual of
    the first half-sweep's blocks (MR minimises it over each step)."""
    dims = (4, 4, 2, 2)
    op = WilsonClover(gauge_links(dims, 0.35, 93), -0.3, 1.2)
    nd = NDOperator(op, 0.05, 0.12)
    eta = doublet(dims, 94)
    from oracle.mg import block_colour
    blk = (2, 2, 2, 2)
    mask0 = (block_colour(dims, blk) == 0).to(torch.float64)[..., None]
    prev = norm(mask0 * eta)
    for steps in range(1, 6):
        # one sweep = colour 0 then colour 1; look at colour 0's residual after its own half-sweep
        z = sap_doublet(nd, mask0 * eta, blk, 1, steps)
        res = norm(mask0 * (mask0 * eta - nd.apply(mask0 * z)))
        assert res <= prev * (1 + 1e-12)
        prev = res
