"""Pins of the oracle pseudofermion force: S_f(phi = D xi) = ||xi||^2
exactly; central finite differences of S_f along random su(3) directions
on 4^4 with dense LU solves; gauge covariance F -> G F G^dag."""
import numpy as np
import pytest
import torch

from lattice_inputs import gauge_links, gaussian_spinor, gell_mann, su3_algebra_coeffs, random_gauge_transform
from oracle.dirac import WilsonClover, spinor_to_field, CDT, dag, lshift
from oracle.force import action_and_force, directional_derivative

DIMS = (4, 4, 4, 4)
M0, CSW, MU = -0.25, 1.6, 0.05


def dense_solver(U):
    op = WilsonClover(U, M0, CSW)
    cache = {}

    def solve(b, mu):
        if mu not in cache:
            cache[mu] = torch.linalg.lu_factor(op.dense(mu))
        LU, piv = cache[mu]
        return torch.linalg.lu_solve(LU, piv, b.reshape(-1, 1)).reshape(b.shape)
    return solve


def action(U, phi):
    op = WilsonClover(U, M0, CSW)
    M = op.dense(MU)
    Y = torch.linalg.solve(M, phi.reshape(-1))
    X = torch.linalg.solve(M.conj().T, Y)
    return float((phi.reshape(-1).conj() @ X).real)


@pytest.fixture(scope="module")
def setup():
    U = torch.tensor(gauge_links(DIMS, 0.35, 61))
    xi = spinor_to_field(gaussian_spinor(DIMS, 62)[0])
    op = WilsonClover(U, M0, CSW)
    phi = op.apply(xi, MU)
    S, F, X, Y = action_and_force(U, M0, CSW, MU, phi, dense_solver(U))
    return U, xi, phi, S, F


def test_action_of_d_xi(setup):
    U, xi, phi, S, F = setup
    assert abs(S - float(torch.sum(xi.conj() * xi).real)) < 1e-10 * S


def test_force_in_su3(setup):
    F = setup[4]
    assert (F + dag(F)).abs().max() < 1e-14
    assert torch.diagonal(F, dim1=-2, dim2=-1).sum(-1).abs().max() < 1e-13
    assert F.abs().max() > 1e-3


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_force_finite_difference(setup, seed):
    U, xi, phi, S, F = setup
    lam = torch.tensor(gell_mann())
    c = torch.tensor(su3_algebra_coeffs(DIMS, 63 + seed))
    omega = torch.einsum("...a,aij->...ij", c.to(CDT), 0.5j * lam)   # sum_a w^a T^a
    h = 1e-5
    Up = torch.linalg.matrix_exp(h * omega) @ U
    Um = torch.linalg.matrix_exp(-h * omega) @ U
    fd = (action(Up, phi) - action(Um, phi)) / (2 * h)
    an = directional_derivative(F, omega)
    assert abs(fd - an) < 1e-7 * abs(an) + 1e-6


def test_force_gauge_covariance(setup):
    U, xi, phi, S, F = setup
    G = torch.tensor(random_gauge_transform(DIMS, 64))
    UG = torch.stack([G @ U[m] @ dag(lshift(G, m, 1)) for m in range(4)])
    phiG = torch.einsum("...ab,...sb->...sa", G, phi.reshape(*phi.shape[:-1], 4, 3)).reshape(phi.shape)
    S2, F2, _, _ = action_and_force(UG, M0, CSW, MU, phiG, dense_solver(UG))
    assert abs(S2 - S) < 1e-10 * S
    assert (F2 - G @ F @ dag(G)).abs().max() < 1e-11
