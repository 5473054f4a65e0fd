"""A small HMC driver for the N_f = 2 twisted-mass clover theory (Sec. 2):
the determinant split by one Hasenbusch mass shift (Eq. (3) with one
ratio), a nested second-order minimal-norm integrator with the gauge action
on the innermost time scale and the fermion monomials outside it (the
heavier one inside the lighter one), the energy violation dH, the
Metropolis test, and the setup update of the multigrid hierarchy along the
trajectory (one setup iteration whenever the force at the physical mass is
computed; the paper updates it at every inversion at that mass).

Every field operation runs in the library: the solves, the fermion and
gauge forces, the momentum and link updates and the kinetic energy.  This
module orders the calls; the random numbers (momenta, pseudofermion
sources) are inputs the caller draws.

Monomials, with Q = Gamma5 D(0) Hermitian and D(m) D(m)^dag =
Gamma5 (Q^2 + m^2) Gamma5 (mu1 = mu + rho):
  ratio  S_r = phi_r^dag D(mu1) D(mu1)^dag (D(mu) D(mu)^dag)^-1 phi_r
             = |phi_r|^2 + (mu1^2 - mu^2) phi_r^dag (D(mu) D(mu)^dag)^-1 phi_r,
         heat bath phi_r = D(mu) D(mu1)^-1 xi_r (then S_r = |xi_r|^2);
  heavy  S_h = phi_h^dag (D(mu1) D(mu1)^dag)^-1 phi_h, heat bath phi_h = D(mu1) xi_h;
  gauge  S_g = beta sum (1 - Re tr P / 3).
Equations of motion for U -> exp(t P) U with P = sum_a p^a T^a:
dU/dt = P U, dP/dt = -F (F the force in the library's convention).
"""
from __future__ import annotations

import math

import torch

from . import binding as b

LAMBDA_2MN = 0.1931833275037836   # minimal-norm second-order integrator


class HMC:
    def __init__(self, solver: b.Solver, U: torch.Tensor, kappa: float, csw: float, mu: float, rho: float,
                 beta: float, steps=(4, 2, 4), tau: float = 1.0, tol: float = 1e-12, setup_iters: int = 1):
        """steps: integration steps of the (ratio, heavy, gauge) time scales,
        outermost first; the inner scales take steps[k] per step of the one
        outside them."""
        self.s = solver
        self.U = U
        self.kappa, self.csw = kappa, csw
        self.mu, self.mu1 = mu, mu + rho
        self.beta = beta
        self.steps = tuple(steps)
        self.tau = tau
        self.tol = tol
        self.setup_iters = setup_iters
        self.F = torch.empty_like(U)
        self.phi_r = None
        self.phi_h = None
        self.links_in_solver = False
        self.iterated = False
        self.force_calls = [0, 0, 0]

    # ---------------------------------------------------------- plumbing
    def _sync_links(self, physical: bool):
        """The solver's links and hierarchy follow U: after the links moved,
        a setup update rebuilds P and D_c on them, with one setup iteration
        before the first physical-mass force (none before a heavier one)."""
        if not self.links_in_solver or (physical and not self.iterated):
            self.s.setup_update(self.U, self.setup_iters if physical else 0)
            self.links_in_solver = True
            self.iterated = physical

    def _links_moved(self):
        self.links_in_solver = False
        self.iterated = False

    # ---------------------------------------------------------- monomials
    def heatbath(self, xi_r: torch.Tensor, xi_h: torch.Tensor):
        """Pseudofermions from Gaussian sources [1][T][Z][Y][X][4][3]."""
        self._sync_links(True)
        y = torch.empty_like(xi_r)
        self.s.solve(xi_r, y, [self.mu1], tol=self.tol)
        self.phi_r = torch.empty_like(xi_r)
        self.s.apply(b.OP_D64, 0, y, self.phi_r, [self.mu])
        self.phi_h = torch.empty_like(xi_h)
        self.s.apply(b.OP_D64, 0, xi_h, self.phi_h, [self.mu1])

    def action_force(self, level: int, with_force: bool = True):
        """(S, F) of the monomial on time scale `level` (0 ratio, 1 heavy,
        2 gauge); F is written into self.F."""
        self.force_calls[level] += 1
        if level == 2:
            return self.s.gauge_force(self.U, self.beta, self.F), self.F
        if level == 1:
            self._sync_links(False)
            S, _ = self.s.force_at(self.phi_h, self.mu1, self.F, tol=self.tol)
            return S, self.F
        self._sync_links(True)
        Sf, _ = self.s.force_at(self.phi_r, self.mu, self.F, tol=self.tol)
        c = self.mu1 ** 2 - self.mu ** 2
        self.F.mul_(c)
        phi2 = float(torch.linalg.vector_norm(self.phi_r) ** 2)
        return phi2 + c * Sf, self.F

    def energy(self, P: torch.Tensor):
        parts = {"kinetic": self.s.md_kinetic(P)}
        for lv, name in ((0, "ratio"), (1, "heavy"), (2, "gauge")):
            parts[name] = self.action_force(lv)[0]
        parts["H"] = sum(parts.values())
        return parts

    # ---------------------------------------------------------- integrator
    def _kick(self, level: int, P: torch.Tensor, c: float):
        _, F = self.action_force(level)
        self.s.md_update_momenta(P, F, -c)

    def _integrate(self, level: int, P: torch.Tensor, eps: float):
        n = self.steps[level]
        h = eps / n
        lam = LAMBDA_2MN
        for _ in range(n):
            self._kick(level, P, lam * h)
            self._inner(level, P, 0.5 * h)
            self._kick(level, P, (1.0 - 2.0 * lam) * h)
            self._inner(level, P, 0.5 * h)
            self._kick(level, P, lam * h)

    def _inner(self, level: int, P: torch.Tensor, dt: float):
        if level + 1 < len(self.steps):
            self._integrate(level + 1, P, dt)
        else:
            self.s.md_update_links(self.U, P, dt)
            self._links_moved()

    def trajectory(self, P: torch.Tensor):
        """Integrate (U, P) over tau in place; returns the energies before
        and after (the pseudofermions stay fixed)."""
        e0 = self.energy(P)
        self._integrate(0, P, self.tau)
        e1 = self.energy(P)
        return e0, e1

    @staticmethod
    def accept(dH: float, uniform: float) -> bool:
        """Metropolis: accept with probability min(1, exp(-dH))."""
        return uniform < math.exp(-dH) if dH > 0 else True
