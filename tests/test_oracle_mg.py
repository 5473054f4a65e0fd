"""Pins of the oracle DD-alpha-AMG components (Sec. 1.1, Eq. (1)):
P^dag P = I and Gamma5 P = P Gamma5,c; D_c = P^dag D P on random vectors,
D_c^dag = Gamma5,c D_c Gamma5,c; D_c(mu) - D_c(0) = i mu Gamma5,c; MR against
a brute-force dense block MR; SAP with exact block solves; the exactly
resolved case (square unitary P) converging in one FGMRES step; FGMRES
against dense solves; the two-step and shifted-system identities."""
import math

import numpy as np
import pytest
import torch

from lattice_inputs import gauge_links, gaussian_spinor, workload, load_m0
from oracle.dirac import WilsonClover, spinor_to_field, norm, CDT
from oracle import mg

D44 = (4, 4, 4, 4)


def rnd(dims, seed, dof=12, n=None):
    v = torch.as_tensor(gaussian_spinor(dims, seed, n=1 if n is None else n, dof=(dof,)))
    return v[0] if n is None else v


@pytest.fixture(scope="module")
def op44():
    return WilsonClover(gauge_links(D44, 0.35, 41), -0.3, 1.4)


@pytest.fixture(scope="module")
def coarse_setup(op44):
    agg = (2, 2, 2, 2)
    V = rnd(D44, 42, n=5)
    P = mg.build_prolongation(V, agg, D44, 12)
    return P, mg.galerkin(op44, P)


def test_prolongation_orthonormal_and_gamma5(coarse_setup):
    P, _ = coarse_setup
    G = torch.einsum("...ki,...kj->...ij", P.Q.conj(), P.Q)
    assert (G - torch.eye(P.nv, dtype=CDT)).abs().max() < 1e-14
    # Gamma5 P = P Gamma5,c on random coarse vectors
    e = rnd(P.coarse_dims, 3, dof=2 * P.nv)
    g5 = mg.gamma5_dof(12)
    g5c = mg.gamma5_dof(2 * P.nv)
    assert norm(g5 * P.prolong(e) - P.prolong(g5c * e)) < 1e-13 * norm(e)
    # P^dag P = I as operators
    assert norm(P.restrict(P.prolong(e)) - e) < 1e-13 * norm(e)


def test_gram_schmidt_span_and_triangular():
    """Q R = V per block with R upper triangular, positive real diagonal."""
    V = rnd(D44, 5, n=4)
    Q = mg.block_gram_schmidt(V, (2, 2, 2, 2))
    vb = mg.to_blocks(V, (2, 2, 2, 2), True).movedim(0, -1)
    R = torch.einsum("...ki,...kj->...ij", Q.conj(), vb)
    assert (Q @ R - vb).abs().max() < 1e-13
    low = torch.tril(R, diagonal=-1)
    assert low.abs().max() < 1e-13
    d = torch.diagonal(R, dim1=-2, dim2=-1)
    assert d.imag.abs().max() < 1e-13 and d.real.min() > 0


def test_galerkin_definition(op44, coarse_setup):
    P, Dc = coarse_setup
    e = rnd(P.coarse_dims, 7, dof=2 * P.nv)
    for mu in (0.0, 0.05):
        lhs = Dc.apply(e, mu)
        rhs = P.restrict(op44.apply(P.prolong(e), mu))
        assert norm(lhs - rhs) < 1e-13 * norm(lhs)


def test_coarse_gamma5_hermiticity(coarse_setup):
    _, Dc = coarse_setup
    M = Dc.dense(0.0).numpy()
    g5 = np.tile(mg.gamma5_dof(Dc.dof).numpy(), int(np.prod(Dc.dims)))
    assert np.abs(M.conj().T - g5[:, None] * M * g5[None, :]).max() < 1e-13
    # backward block = Gamma5,c (forward block of the neighbour)^dag Gamma5,c
    g5c = mg.gamma5_dof(Dc.dof)
    for m in range(4):
        fwd_nb = mg.shift(Dc.F[m], m, -1, xaxis=-3)
        expect = g5c[:, None] * fwd_nb.conj().transpose(-1, -2) * g5c[None, :]
        assert (Dc.B[m] - expect).abs().max() < 1e-13


def test_coarse_twisted_mass(coarse_setup):
    _, Dc = coarse_setup
    mu = 0.37
    d = Dc.dense(mu) - Dc.dense(0.0)
    g5 = torch.tensor(np.tile(mg.gamma5_dof(Dc.dof).numpy(), int(np.prod(Dc.dims))))
    assert (d - 1j * mu * torch.diag(g5).to(CDT)).abs().max() < 1e-14


def test_coarse_extent_two_neighbours(op44):
    """2^4 aggregates on 4^4 give a 2^4 coarse lattice where y+mu = y-mu:
    both blocks are kept and applied; the result is still exact Galerkin."""
    P = mg.build_prolongation(rnd(D44, 8, n=3), (2, 2, 2, 2), D44, 12)
    Dc = mg.galerkin(op44, P)
    e = rnd(P.coarse_dims, 9, dof=6)
    assert norm(Dc.apply(e, 0.1) - P.restrict(op44.apply(P.prolong(e), 0.1))) < 1e-13 * norm(e) * 10


def _dense_block_mr(op, r, blk, colour, steps, mu):
    """Brute force: extract every block's dense matrix and run MR in numpy."""
    M = op.dense(mu).numpy()
    dims = op.dims
    lx, ly, lz, lt = dims
    col = mg.block_colour(dims, blk).numpy()
    x = mg.coords(dims)
    bid = sum((x[m] // blk[m]).numpy() * int(np.prod([dims[k] // blk[k] for k in range(m)]))
              for m in range(4))
    rv = r.numpy().reshape(-1)
    e = np.zeros_like(rv)
    for b in np.unique(bid[col == colour]):
        sites = np.nonzero((bid == b).reshape(-1))[0]
        idx = (sites[:, None] * 12 + np.arange(12)).reshape(-1)
        A = M[np.ix_(idx, idx)]
        rho = rv[idx].copy()
        eb = np.zeros_like(rho)
        for _ in range(steps):
            q = A @ rho
            a = np.vdot(q, rho) / np.vdot(q, q)
            eb += a * rho
            rho -= a * q
        e[idx] = eb
    return e.reshape(r.shape)


def test_mr_block_solve_matches_dense(op44):
    blk = (2, 2, 2, 2)
    mu = 0.05
    colour = mg.block_colour(D44, blk)
    mask = (colour == 1).to(torch.float64)[..., None]
    r = mask * rnd(D44, 10)
    e, rho = mg.mr_block_solve(op44, r, mask, blk, 4, mu)
    e_ref = _dense_block_mr(op44, r, blk, 1, 4, mu)
    assert np.abs(e.numpy() - e_ref).max() < 1e-13
    # rho is the block residual r - D_B e
    assert norm(rho - (r - mask * op44.apply(e, mu))) < 1e-13 * norm(r)


def test_mr_residual_monotone(op44):
    blk = (2, 2, 2, 2)
    mask = (mg.block_colour(D44, blk) == 0).to(torch.float64)[..., None]
    r = mask * rnd(D44, 11)
    prev = norm(r)
    for s in range(1, 8):
        _, rho = mg.mr_block_solve(op44, r, mask, blk, s, 0.02)
        assert norm(rho) <= prev * (1 + 1e-14)
        prev = norm(rho)


def test_sap_exact_blocks_zero_colour_residual(op44):
    """With exact block solves, after a colour's half-sweep the residual on
    that colour's blocks vanishes."""
    blk = (2, 2, 2, 2)
    mu = 0.03
    M = op44.dense(mu)

    def exact(r, mask):
        # blocks of one colour decouple; solving the masked system solves each block
        m = mask.expand_as(r).reshape(-1).bool()
        idx = torch.nonzero(m).squeeze(1)
        A = M[idx][:, idx]
        e = torch.zeros(r.numel(), dtype=CDT)
        e[idx] = torch.linalg.solve(A, r.reshape(-1)[idx])
        return e.reshape(r.shape)

    eta = rnd(D44, 12)
    colour = mg.block_colour(D44, blk)
    # one colour-0 half sweep by hand through the oracle with sweeps=1 then colour 1
    mask0 = (colour == 0).to(torch.float64)[..., None]
    z = torch.zeros_like(eta)
    r = mask0 * (eta - op44.apply(z, mu))
    z = z + exact(r, mask0)
    res = eta - op44.apply(z, mu)
    assert norm(mask0 * res) < 1e-12 * norm(eta)
    # full sap with exact blocks: residual on colour 1 vanishes after the sweep
    zs = mg.sap(op44, eta, torch.zeros_like(eta), mu, blk, 1, 0, block_solver=exact)
    mask1 = (colour == 1).to(torch.float64)[..., None]
    assert norm(mask1 * (eta - op44.apply(zs, mu))) < 1e-12 * norm(eta)


def test_sap_single_block_exact_is_inverse(op44):
    mu = 0.03
    M = op44.dense(mu)
    exact = lambda r, mask: torch.linalg.solve(M, (mask * r).reshape(-1)).reshape(r.shape)
    eta = rnd(D44, 13)
    z = mg.sap(op44, eta, torch.zeros_like(eta), mu, D44, 1, 0, block_solver=exact)
    assert norm(op44.apply(z, mu) - eta) < 1e-12 * norm(eta)


def test_fgmres_matches_dense(op44):
    mu = 0.05
    b = rnd(D44, 14)
    res = mg.fgmres(lambda v: op44.apply(v, mu), b, 1e-12, 40, 2000)
    x_ref = torch.linalg.solve(op44.dense(mu), b.reshape(-1)).reshape(b.shape)
    assert res.converged
    assert norm(op44.apply(res.x, mu) - b) / norm(b) < 2e-12
    assert norm(res.x - x_ref) / norm(x_ref) < 1e-9
    # implicit residual history agrees with the true residual at the end
    assert abs(res.resid[-1] - norm(op44.apply(res.x, mu) - b) / norm(b)) < 1e-12


def test_fgmres_with_identity_preconditioner_is_gmres(op44):
    mu = 0.05
    b = rnd(D44, 15)
    a = lambda v: op44.apply(v, mu)
    r1 = mg.fgmres(a, b, 1e-8, 20, 60)
    r2 = mg.fgmres(a, b, 1e-8, 20, 60, apply_m=lambda v: v.clone())
    assert r1.iters == r2.iters
    assert norm(r1.x - r2.x) < 1e-12 * norm(r1.x)


def test_exactly_resolved_case_one_iteration():
    """Aggregates of one site with N_v = 6: P is square and unitary, so the
    coarse correction of Eq. (1) with an exact coarse solve removes the whole
    error and FGMRES converges in one step."""
    dims = (2, 2, 2, 4)
    op = WilsonClover(gauge_links(dims, 0.35, 51), -0.2, 1.2)
    mu = 0.04
    p = mg.MGParams(nlevels=2, agg=((1, 1, 1, 1),), nv=(6,), sap_block=((1, 1, 2, 2),),
                    setup_iters=0, coarsest_tol=1e-14, coarsest_maxiter=400)
    H = mg.Hierarchy(op, p, mu)
    H.setup(mg.setup_vectors(p, dims, 52))
    b = rnd(dims, 53)
    res = H.solve(b, 1e-10, restart=10, maxiter=10)
    assert res.converged and res.iters == 1
    assert norm(op.apply(res.x, mu) - b) / norm(b) < 1e-10


def test_shifted_identity(op44):
    """D(mu) D(mu)^dag + sigma = D(mu') D(mu')^dag, mu' = sqrt(mu^2 + sigma)."""
    mu, sigma = 0.02, 0.3
    mup = math.sqrt(mu * mu + sigma)
    v = rnd(D44, 16)
    lhs = op44.apply(op44.apply_dag(v, mu), mu) + sigma * v
    rhs = op44.apply(op44.apply_dag(v, mup), mup)
    assert norm(lhs - rhs) < 1e-12 * norm(lhs)


@pytest.fixture(scope="module")
def c1_hierarchy():
    w = workload("c1")
    m0 = load_m0()["c1"]
    op = WilsonClover(gauge_links(w.dims, w.eps, w.seeds["links"]), m0, w.csw)
    p = mg.MGParams(nlevels=2, agg=w.agg, nv=w.nv, sap_block=w.sap_block,
                    setup_iters=w.setup_iters, mr_steps=w.mr_steps)
    H = mg.Hierarchy(op, p, w.mu)
    H.setup(mg.setup_vectors(p, w.dims, w.seeds["testvec"]))
    return w, op, H


def test_c1_solve_true_residual(c1_hierarchy):
    w, op, H = c1_hierarchy
    b = spinor_to_field(gaussian_spinor(w.dims, w.seeds["source"])[0])
    res = H.solve(b, 1e-10, restart=w.restart)
    assert res.converged
    assert norm(b - op.apply(res.x, w.mu)) / norm(b) <= 1e-10
    assert res.iters < 60


def test_c1_two_step_and_shifted(c1_hierarchy):
    w, op, H = c1_hierarchy
    b = spinor_to_field(gaussian_spinor(w.dims, w.seeds["source"] + 7)[0])
    y = mg.two_step_solve(H, b, w.mu, 1e-11)
    ddy = op.apply_dag(op.apply(y, w.mu), w.mu)
    assert norm(ddy - b) / norm(b) < 1e-8
    sigma = 0.01
    x = mg.shifted_solve(H, b, sigma, w.mu, 1e-11)
    lhs = op.apply(op.apply_dag(x, w.mu), w.mu) + sigma * x
    assert norm(lhs - b) / norm(b) < 1e-8


def test_three_level_exactly_resolved_case_one_iteration():
    """Three levels, both coarsenings square and unitary (one-site aggregates,
    N_v = 6 at each, so 2 N_v equals the dof of the finer site).  The coarsest
    GMRES is run to 1e-14, so the level-1 cycle is an exact inverse of D_c,
    the intermediate FGMRES (preconditioned by that cycle, Sec. 1.1) needs one
    step per call, and the fine FGMRES converges in one iteration.  A wrong
    operator, transfer or sign anywhere in the intermediate branch breaks
    either count."""
    dims = (2, 2, 2, 4)
    op = WilsonClover(gauge_links(dims, 0.35, 61), -0.2, 1.2)
    mu = 0.04
    p = mg.MGParams(nlevels=3, agg=((1, 1, 1, 1), (1, 1, 1, 1)), nv=(6, 6),
                    sap_block=((1, 1, 2, 2), (1, 1, 2, 2)), setup_iters=0,
                    l2_tol=1e-14, l2_restart=10, l2_maxiter=10,
                    coarsest_tol=1e-14, coarsest_maxiter=400)
    H = mg.Hierarchy(op, p, mu)
    H.setup(mg.setup_vectors(p, dims, 62))
    assert len(H.levels) == 2 and H.levels[1].nxt is not None and H.levels[1].nxt.nxt is None
    H.stats = {"coarse_iters": 0, "coarsest_iters": 0}
    b = rnd(dims, 63)
    res = H.solve(b, 1e-10, restart=10, maxiter=10)
    assert res.converged and res.iters == 1
    assert norm(op.apply(res.x, mu) - b) / norm(b) < 1e-10
    # one fine iteration = one intermediate solve, which took a single step
    assert H.stats["coarse_iters"] == 1
    # and the intermediate solve reproduces D_c^-1 on its own
    lvl1 = H.levels[1]
    rc = rnd(lvl1.op.dims, 64, dof=12)
    ec = H.coarse_solve(lvl1, rc, mu)
    assert norm(lvl1.op.apply(ec, mu) - rc) / norm(rc) < 1e-12


def test_setup_iterations_improve_convergence():
    """Quality trend of the adaptive setup (its result is not unique, so
    this is the check the method admits): the outer FGMRES iteration count
    does not grow with the number of setup iterations (0, 1, 3), and three
    iterations at least halve the count of the initial phase alone.

    Input: the 8^4 workload's links with periodic time and m0 = -0.17, where
    SAP alone needs 82 iterations.  With the workload's antiperiodic time the
    lowest momentum keeps |lambda| near sin(pi/8) and SAP alone converges
    in 22 iterations, so no coarse space (random or adapted) can show a
    trend there."""
    w = workload("c1")
    op = WilsonClover(gauge_links(w.dims, w.eps, w.seeds["links"]), -0.17, w.csw, antiperiodic=False)
    mu = 0.001
    b = spinor_to_field(gaussian_spinor(w.dims, w.seeds["source"])[0])
    its = {}
    for n in (0, 1, 3):
        p = mg.MGParams(nlevels=2, agg=w.agg, nv=w.nv, sap_block=w.sap_block,
                        setup_iters=n, mr_steps=w.mr_steps)
        H = mg.Hierarchy(op, p, mu)
        H.setup(mg.setup_vectors(p, w.dims, w.seeds["testvec"]))
        r = H.solve(b, 1e-10, restart=w.restart)
        assert r.converged
        assert norm(b - op.apply(r.x, mu)) / norm(b) <= 1e-10
        its[n] = r.iters
    print("outer iterations by setup iterations:", its)
    assert its[0] >= its[1] >= its[3]
    assert 2 * its[3] <= its[0]
