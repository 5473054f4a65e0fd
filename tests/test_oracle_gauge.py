"""Pins of the oracle gauge action and force: zero at unit links; the
closed form of links in a U(1) subgroup (diag(e^{i phi}, e^{-i phi}, 1),
where Re tr P = 2 cos(Theta) + 1 with Theta the plaquette's phase sum);
gauge invariance; the force against central finite differences along
random su(3) directions."""
import numpy as np
import torch

from lattice_inputs import gauge_links, random_gauge_transform, su3_algebra_coeffs, gell_mann
from oracle.dirac import CDT, dag
from oracle import gauge

DIMS = (4, 4, 4, 6)
BETA = 5.6


def test_unit_links_zero_action_and_force():
    U = torch.eye(3, dtype=CDT).expand(4, 6, 4, 4, 4, 3, 3).clone()
    assert float(gauge.action(U, BETA)) == 0.0
    assert float(gauge.force(U, BETA).abs().max()) == 0.0


def test_u1_subgroup_closed_form():
    rng = np.random.default_rng(81)
    lx, ly, lz, lt = DIMS
    phi = torch.tensor(rng.uniform(-np.pi, np.pi, size=(4, lt, lz, ly, lx)))
    U = torch.zeros(4, lt, lz, ly, lx, 3, 3, dtype=CDT)
    U[..., 0, 0] = torch.exp(1j * phi)
    U[..., 1, 1] = torch.exp(-1j * phi)
    U[..., 2, 2] = 1.0
    S = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            th = phi[mu] + torch.roll(phi[nu], -1, dims=3 - mu) - torch.roll(phi[mu], -1, dims=3 - nu) - phi[nu]
            S += float(torch.sum(2.0 / 3.0 * (1.0 - torch.cos(th))))
    assert abs(float(gauge.action(U, 1.0)) - S) < 1e-10 * S


def test_gauge_invariance():
    U = torch.tensor(gauge_links(DIMS, 0.5, 82))
    G = torch.tensor(random_gauge_transform(DIMS, 83))
    UG = torch.stack([G @ U[m] @ dag(torch.roll(G, -1, dims=3 - m)) for m in range(4)])
    assert abs(float(gauge.action(UG, BETA) - gauge.action(U, BETA))) < 1e-10 * float(gauge.action(U, BETA))


def test_force_matches_finite_differences():
    U = torch.tensor(gauge_links(DIMS, 0.5, 84))
    F = gauge.force(U, BETA)
    lam = torch.tensor(gell_mann())
    for seed in (85, 86, 87):
        c = torch.tensor(su3_algebra_coeffs(DIMS, seed))           # [4, T, Z, Y, X, 8]
        w = torch.einsum("...a,aij->...ij", c.to(CDT), 0.5j * lam)
        h = 1e-5
        Sp = float(gauge.action(torch.matrix_exp(h * w) @ U, BETA))
        Sm = float(gauge.action(torch.matrix_exp(-h * w) @ U, BETA))
        fd = (Sp - Sm) / (2 * h)
        an = float(-2.0 * torch.einsum("...ij,...ji->", F, w).real)
        assert abs(fd - an) < 1e-6 * abs(an)
