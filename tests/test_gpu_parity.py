"""GPU parity of every step of the hot path against the CPU oracle, through
the C ABI: fine stencil (FP64, FP32), clover, restriction/prolongation,
block Gram-Schmidt, Galerkin D_c, coarse operator, SAP, one multigrid
cycle, and full solves (2 and 3 levels, FP64 and mixed precision)."""
import math

import numpy as np
import pytest
import torch

from lattice_inputs import workload, load_m0
from oracle.dirac import WilsonClover, norm
from oracle import mg
from tests.gpu_common import DEV, links, spinors, kappa_of, rel, field, to_dev, maxabs_rel

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c1():
    w = workload("c1")
    m0 = load_m0()["c1"]
    U, Ud = links(w.dims, w.eps, w.seeds["links"])
    op = WilsonClover(U, m0, w.csw)
    return w, m0, U, Ud, op


def make_solver(w, nlevels=2, precision=tm.FP64, **kw):
    p = dict(nlevels=nlevels, agg=w.agg, nv=w.nv, setup_iters=w.setup_iters, init_smooth=w.init_smooth,
             sap_sweeps=w.sap_sweeps, mr_steps=w.mr_steps, restart=w.restart, precision=precision)
    if nlevels == 3:
        p["sap_block1"] = w.sap_block[1]
    p.update(kw)
    return tm.Solver(w.dims, tm.default_params(**p))


def test_stencil_fp64_fp32(c1):
    w, m0, U, Ud, op = c1
    say("stencil parity c1", w.dims)
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_FP32)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    psi, psid = spinors(w.dims, 77, 3)
    mus = [w.mu, -0.03, 0.0]
    out = torch.empty_like(psid)
    s.apply(tm.OP_D64, 0, psid, out, mus)
    ref = torch.stack([op.apply(field(psi[r]), mus[r]) for r in range(3)])
    assert rel(field(out.cpu()), ref) < 1e-13
    s.apply(tm.OP_D32, 0, psid, out, mus)
    assert rel(field(out.cpu()), ref) < 2e-6


def test_stencil_rectangular_lattice():
    dims = (8, 4, 4, 16)
    say("stencil parity", dims)
    U, Ud = links(dims, 0.4, 91)
    op = WilsonClover(U, -0.2, 1.3)
    p = tm.default_params(nlevels=0, setup_iters=0, init_smooth=0)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(-0.2), 1.3, 0.05)
    psi, psid = spinors(dims, 92, 2)
    out = torch.empty_like(psid)
    s.apply(tm.OP_D64, 0, psid, out, [0.05, 0.2])
    ref = torch.stack([op.apply(field(psi[0]), 0.05), op.apply(field(psi[1]), 0.2)])
    assert rel(field(out.cpu()), ref) < 1e-13
    # periodic time: no sign on the boundary hops
    op_p = WilsonClover(U, -0.2, 1.3, antiperiodic=False)
    sp = tm.Solver(dims, p, antiperiodic=False)
    sp.setup(Ud, kappa_of(-0.2), 1.3, 0.05)
    sp.apply(tm.OP_D64, 0, psid, out, [0.05, 0.05])
    assert rel(field(out.cpu())[0], op_p.apply(field(psi[0]), 0.05)) < 1e-13


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-11), ("mixed", 1e-5)])
def test_sap_blocks_spanning_a_direction(precision, bar):
    """SAP on a lattice whose 4^4 blocks span two directions (x and z: one
    block there, so the periodic hop stays inside the block) and cut the
    other two, against the oracle's SAP; bars as for the SAP tests on 8^4."""
    dims = (4, 8, 4, 8)
    U, Ud = links(dims, 0.35, 93)
    m0, csw, mus = -0.2, 1.3, [0.05, -0.1]
    op = WilsonClover(U, m0, csw)
    psi, psid = spinors(dims, 94, 2)
    say("SAP parity", dims, precision)
    p = tm.default_params(nlevels=1, agg=[[4, 4, 4, 4], [2, 2, 2, 2]], setup_iters=0, init_smooth=0,
                          sap_sweeps=[4, 2], mr_steps=4, precision=tm.FP64 if precision == "fp64" else tm.MIXED)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(m0), csw, 0.05)
    out = torch.empty_like(psid)
    s.apply(tm.OP_SAP, 0, psid, out, mus)
    worst = 0.0
    for r, mu in enumerate(mus):
        eta = field(psi[r])
        ref = mg.sap(op, eta, torch.zeros_like(eta), mu, (4, 4, 4, 4), 4, 4)
        worst = max(worst, rel(field(out.cpu()[r]), ref), maxabs_rel(field(out.cpu()[r]), ref))
    say(f"  worst rel. difference {worst:.2e}")
    assert worst < bar
    s.close()


@pytest.fixture(scope="module")
def injected_c1(c1):
    """2-level hierarchy built from injected test vectors, no smoothing or
    setup iterations: P and D_c are then unique."""
    w, m0, U, Ud, op = c1
    s = make_solver(w, setup_iters=0, init_smooth=0)
    tv, tvd = spinors(w.dims, 4321, w.nv[0])
    s.set_test_vectors(0, tvd)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    P = mg.build_prolongation(field(tv), w.agg[0], w.dims, 12)
    Dc = mg.galerkin(op, P)
    return s, P, Dc


def test_prolongation_and_galerkin(c1, injected_c1):
    w, m0, U, Ud, op = c1
    s, P, Dc = injected_c1
    say("P / D_c parity c1")
    nv = w.nv[0]
    lx, ly, lz, lt = w.dims
    Pg = torch.empty((nv, lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device=DEV)
    s.export(0, 0, Pg)
    # oracle P as nv canonical fields: column (s, i) lives in field i, chirality s
    e = torch.zeros(nv, *P.coarse_dims[::-1], 2 * nv, dtype=torch.complex128)
    ref = []
    for i in range(nv):
        ei = torch.zeros(*P.coarse_dims[::-1], 2 * nv, dtype=torch.complex128)
        ei[..., i] = 1.0
        ei[..., nv + i] = 1.0
        ref.append(P.prolong(ei))
    ref = torch.stack(ref)
    assert rel(field(Pg.cpu()), ref) < 1e-12
    Vc, d = s.level_info(1)
    D = torch.empty((Vc, 9, d, d), dtype=torch.complex128, device=DEV)
    s.export(1, 1, D)
    D = D.cpu().transpose(-1, -2)   # [col][row] -> [row][col]
    lxc, lyc, lzc, ltc = P.coarse_dims
    Sref = Dc.S.reshape(-1, d, d)
    assert rel(D[:, 0], Sref) < 1e-12
    for m in range(4):
        assert rel(D[:, 1 + 2 * m], Dc.F[m].reshape(-1, d, d)) < 1e-12
        assert rel(D[:, 2 + 2 * m], Dc.B[m].reshape(-1, d, d)) < 1e-12


# Mixed precision with bf16 storage: P is the oracle's block Gram-Schmidt
# rounded to bf16, and D_c is the library's FP32 Galerkin product (its
# projection on the matrix cores) from that rounded P, rounded to bf16.
# Checked against the oracle's FP64 product from the library's own rounded
# P.  Bars from the arithmetic: bf16 rounding (2^-9 relative per entry)
# dominates both.
@pytest.mark.parametrize("nv", [24, 16])
def test_prolongation_and_galerkin_mixed_bf16(c1, nv):
    w, m0, U, Ud, op = c1
    say("P / D_c parity c1, mixed bf16, nv", nv)
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_BF16, setup_iters=0, init_smooth=0, nv=(nv, 0))
    tv, tvd = spinors(w.dims, 4331 + nv, nv)
    s.set_test_vectors(0, tvd)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    lx, ly, lz, lt = w.dims
    Pg = torch.empty((nv, lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device=DEV)
    s.export(0, 0, Pg)
    Vr = field(Pg.cpu())                                   # the library's rounded P as nv fields
    P64 = mg.build_prolongation(field(tv), w.agg[0], w.dims, 12)
    Q = mg.to_blocks(Vr, w.agg[0], True).movedim(0, -1).contiguous()
    Pr = mg.Prolongation(Q, w.agg[0], w.dims, 12)
    err_p = rel(Pr.Q, P64.Q)
    say(f"  P vs FP64 Gram-Schmidt: {err_p:.2e}")
    assert err_p < 4e-3
    Dc = mg.galerkin(op, Pr)
    Vc, d = s.level_info(1)
    D = torch.empty((Vc, 9, d, d), dtype=torch.complex128, device=DEV)
    s.export(1, 1, D)
    D = D.cpu().transpose(-1, -2)
    errs = [rel(D[:, 0], Dc.S.reshape(-1, d, d))]
    for m in range(4):
        errs.append(rel(D[:, 1 + 2 * m], Dc.F[m].reshape(-1, d, d)))
        errs.append(rel(D[:, 2 + 2 * m], Dc.B[m].reshape(-1, d, d)))
    say(f"  D_c blocks, worst rel. difference {max(errs):.2e}")
    assert max(errs) < 4e-3
    # elementwise, per stored block: bf16 keeps 8 significant bits, so each
    # entry is within 2^-9 of itself and 2^-8 of its block's largest entry
    refs = [Dc.S.reshape(-1, d, d)] + [t for m in range(4) for t in (Dc.F[m].reshape(-1, d, d),
                                                                       Dc.B[m].reshape(-1, d, d))]
    worst_blk = 0.0
    for b, ref in enumerate(refs):
        dev_ = (D[:, b] - ref).abs().amax(dim=(-1, -2))
        scale = ref.abs().amax(dim=(-1, -2))
        worst_blk = max(worst_blk, float((dev_ / scale).max()))
    say(f"  D_c elementwise, worst deviation over the block's largest entry {worst_blk:.2e} (bound 2^-8)")
    assert worst_blk <= 2.0 ** -8
    # batched transfers (20 right-hand sides: the matrix-core kernels, one
    # full group of 16 and a ragged one; 4: the vector-ALU kernels; then
    # each family forced to the other variant through the variant table:
    # 20 on the vector ALU, 1 on the matrix cores) against the oracle's
    # FP64 P^dag and P with the library's rounded P.  Bar: the two-part
    # bf16 split keeps each input to 4e-6.
    V = math.prod(w.dims)
    for nrhs, forced in ((20, None), (4, None), (20, 0), (1, 1)):
        psi, psid = spinors(w.dims, 57 + nrhs, nrhs)
        try:
            if forced is not None:
                tm.tune_set(tm.TUNE_RESTRICT0, nv, V, nrhs, forced)
                tm.tune_set(tm.TUNE_PROLONG0, nv, V, nrhs, forced)
            rc = torch.empty((nrhs, Vc, d), dtype=torch.complex128, device=DEV)
            s.apply(tm.OP_RESTRICT, 0, psid, rc)
            back = torch.empty_like(psid)
            s.apply(tm.OP_PROLONG, 1, rc, back)
        finally:
            tm.tune_clear()
        ref = torch.stack([Pr.restrict(field(psi[r])).reshape(Vc, d) for r in range(nrhs)])
        err_r = rel(rc.cpu(), ref)
        refp = torch.stack([Pr.prolong(rc.cpu()[r].reshape(*Pr.coarse_dims[::-1], d)) for r in range(nrhs)])
        err_p = rel(field(back.cpu()), refp)
        el_r, el_p = maxabs_rel(rc.cpu(), ref), maxabs_rel(field(back.cpu()), refp)
        say(f"  {nrhs} RHS (variant {forced}): P^dag {err_r:.2e} ({el_r:.2e} elementwise), P {err_p:.2e} "
            f"({el_p:.2e})")
        assert err_r < 2e-5 and err_p < 2e-5 and el_r < 2e-5 and el_p < 2e-5


def test_transfers_and_coarse_operator(c1, injected_c1):
    w, m0, U, Ud, op = c1
    s, P, Dc = injected_c1
    say("restrict / prolong / D_c parity c1")
    Vc, d = s.level_info(1)
    psi, psid = spinors(w.dims, 55, 2)
    rc = torch.empty((2, Vc, d), dtype=torch.complex128, device=DEV)
    s.apply(tm.OP_RESTRICT, 0, psid, rc)
    ref = torch.stack([P.restrict(field(psi[r])).reshape(Vc, d) for r in range(2)])
    assert rel(rc.cpu(), ref) < 1e-12
    back = torch.empty_like(psid)
    s.apply(tm.OP_PROLONG, 1, rc, back)
    refp = torch.stack([P.prolong(ref[r].reshape(*P.coarse_dims[::-1], d)) for r in range(2)])
    assert rel(field(back.cpu()), refp) < 1e-12
    out = torch.empty_like(rc)
    s.apply(tm.OP_DC, 1, rc, out, [w.mu, -0.2])
    refd = torch.stack([Dc.apply(ref[0].reshape(*P.coarse_dims[::-1], d), w.mu).reshape(Vc, d),
                        Dc.apply(ref[1].reshape(*P.coarse_dims[::-1], d), -0.2).reshape(Vc, d)])
    assert rel(out.cpu(), refd) < 1e-12


def test_sap_fixed_steps(c1):
    """The FP64 fine SAP (k sweeps of MR block solves) against the oracle's
    SAP, two right-hand sides with different mu."""
    w, m0, U, Ud, op = c1
    say("SAP parity c1, FP64")
    s = make_solver(w, setup_iters=0, init_smooth=0)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    psi, psid = spinors(w.dims, 66, 2)
    out = torch.empty_like(psid)
    s.apply(tm.OP_SAP, 0, psid, out, [w.mu, 0.1])
    worst = 0.0
    for r, mu in enumerate([w.mu, 0.1]):
        eta = field(psi[r])
        ref = mg.sap(op, eta, torch.zeros_like(eta), mu, w.sap_block[0], w.sap_sweeps[0], w.mr_steps)
        worst = max(worst, rel(field(out.cpu()[r]), ref))
    say(f"  worst rel. difference {worst:.2e}")
    assert worst < 1e-11


@pytest.mark.parametrize("nrhs,variant", [(1, None), (3, None), (3, 2), (4, 2), (1, 2), (4, 1)])
def test_sap_fixed_steps_fp32(c1, nrhs, variant):
    """The FP32 fine SAP (k sweeps of 4 MR steps per block) against the
    oracle's FP64 SAP, one right-hand side (one workgroup per block) and
    batches with signed per-RHS mu: the batched kernel (variant 1) and the
    kernel with two right-hand sides per workgroup (variant 2; odd counts
    leave a lone last one).  Bar: FP32 rounding through 16 block solves of
    a few hundred FP32 operations each per site, about 1e-6; 1e-5 in l2 and
    elementwise against the field's largest entry."""
    w, m0, U, Ud, op = c1
    say("SAP parity c1, FP32,", nrhs, "RHS, variant", variant)
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_BF16, setup_iters=0, init_smooth=0)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    mus = [w.mu, -0.1, 0.03, 0.2][:nrhs]
    psi, psid = spinors(w.dims, 68 + nrhs, nrhs)
    out = torch.empty_like(psid)
    V = w.dims[0] * w.dims[1] * w.dims[2] * w.dims[3]
    if variant is not None:
        tm.tune_set(tm.TUNE_SAP0, 256, V, nrhs, variant)
    try:
        s.apply(tm.OP_SAP, 0, psid, out, mus)
    finally:
        if variant is not None:
            tm.tune_set(tm.TUNE_SAP0, 256, V, nrhs, -1)
    worst = worst_el = 0.0
    for r, mu in enumerate(mus):
        eta = field(psi[r])
        ref = mg.sap(op, eta, torch.zeros_like(eta), mu, w.sap_block[0], w.sap_sweeps[0], w.mr_steps)
        worst = max(worst, rel(field(out.cpu()[r]), ref))
        worst_el = max(worst_el, maxabs_rel(field(out.cpu()[r]), ref))
    say(f"  worst rel. difference {worst:.2e}, elementwise {worst_el:.2e}")
    assert worst < 1e-5 and worst_el < 1e-5


@pytest.mark.parametrize("prec,bar", [(64, 1e-13), (32, 2e-6)])
def test_schur_operator_parity(c1, prec, bar):
    """The even-odd reduced operator D_ee - D_eo D_oo^-1 D_oe (two parity
    passes, the odd-site clover block solved in the kernel) against the
    oracle's Schur complement with per-site dense inverses, two right-hand
    sides with signed mu; odd outputs are exactly zero.  Bars as for the
    stencil (FP32: the 6x6 elimination adds a few roundings of a
    well-conditioned block)."""
    from oracle.evenodd import SchurOperator
    w, m0, U, Ud, op = c1
    say("Schur operator c1, FP", prec)
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_BF16, setup_iters=0, init_smooth=0)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    psi, psid = spinors(w.dims, 5501, 2)
    out = torch.empty_like(psid)
    mus = [w.mu, -0.05]
    s.apply(tm.OP_SCHUR64 if prec == 64 else tm.OP_SCHUR32, 0, psid, out, mus)
    got = field(out.cpu())
    worst = 0.0
    for r in range(2):
        S = SchurOperator(op, mus[r])
        worst = max(worst, rel(got[r], S.apply(field(psi[r]))))
        assert float((got[r] * S.odd).abs().max()) == 0.0
    say(f"  worst rel. difference {worst:.2e}")
    assert worst < bar


def test_multigrid_cycle(c1, injected_c1):
    w, m0, U, Ud, op = c1
    s, P, Dc = injected_c1
    say("B_MG parity c1")
    psi, psid = spinors(w.dims, 67, 1)
    out = torch.empty_like(psid)
    s.apply(tm.OP_PREC, 0, psid, out)
    p = mg.MGParams(nlevels=2, agg=w.agg, nv=w.nv, sap_block=w.sap_block, setup_iters=0,
                    mr_steps=w.mr_steps, init_smooth=0)
    H = mg.Hierarchy(op, p, w.mu)
    lvl = H.levels[0]
    lvl.P = P
    lvl.nxt = mg.Level(Dc, 1)
    ref = H.precondition(lvl, field(psi[0]), w.mu)
    assert rel(field(out.cpu()[0]), ref) < 1e-9


def test_solve_c1_fp64(c1):
    w, m0, U, Ud, op = c1
    say("solve c1 fp64 2-level")
    s = make_solver(w)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, w.seeds["source"], 1)
    x = torch.empty_like(bd)
    info = s.solve(bd, x, tol=w.tol)
    say("info", info.as_dict())
    assert info.status == 0
    r = norm(field(b[0]) - op.apply(field(x.cpu()[0]), w.mu)) / norm(field(b[0]))
    assert r <= 1e-10
    assert info.outer_iters < 80


def test_solve_c1_mixed_batched(c1):
    w, m0, U, Ud, op = c1
    say("solve c1 mixed bf16 batched")
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_BF16)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, 2011, 3)
    x = torch.empty_like(bd)
    mus = [w.mu, -w.mu, 0.05]
    info = s.solve(bd, x, mus, tol=w.tol)
    say("info", info.as_dict())
    assert info.status == 0
    for r in range(3):
        res = norm(field(b[r]) - op.apply(field(x.cpu()[r]), mus[r])) / norm(field(b[r]))
        assert res <= 1e-10


def test_solve_three_level():
    dims = (8, 8, 8, 16)
    say("solve 3-level", dims)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1234)
    op = WilsonClover(U, m0, 1.6)
    p = tm.default_params(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16), sap_block1=(1, 1, 1, 2),
                          coarsest_iters=50, setup_iters=2)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(m0), 1.6, 0.003)
    b, bd = spinors(dims, 99, 2)
    x = torch.empty_like(bd)
    info = s.solve(bd, x, tol=1e-10)
    say("info", info.as_dict())
    assert info.status == 0
    for r in range(2):
        assert norm(field(b[r]) - op.apply(field(x.cpu()[r]), 0.003)) / norm(field(b[r])) <= 1e-10


def test_solve_shifted(c1):
    w, m0, U, Ud, op = c1
    say("shifted solve c1")
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_FP16)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, 3011, 2)
    x = torch.empty_like(bd)
    sig = [0.0, 0.01]
    info = s.solve_shifted(bd, x, sig, tol=1e-11)
    assert info.status == 0
    for r in range(2):
        xr = field(x.cpu()[r])
        lhs = op.apply(op.apply_dag(xr, w.mu), w.mu) + sig[r] * xr
        assert norm(lhs - field(b[r])) / norm(field(b[r])) < 1e-8


@pytest.fixture(scope="module")
def injected_three_level():
    """3-level hierarchy from injected test vectors on both coarsenings."""
    dims = (8, 8, 8, 16)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1235)
    op = WilsonClover(U, m0, 1.6)
    nv = (12, 16)
    agg = ((4, 4, 4, 4), (2, 2, 2, 2))
    sap1 = (1, 1, 1, 2)
    p = tm.default_params(nlevels=3, agg=agg, nv=nv, sap_block1=sap1, coarsest_iters=50, setup_iters=0,
                          init_smooth=0)
    s = tm.Solver(dims, p)
    tv0, tv0d = spinors(dims, 7001, nv[0])
    s.set_test_vectors(0, tv0d)
    P0 = mg.build_prolongation(field(tv0), agg[0], dims, 12)
    Dc1 = mg.galerkin(op, P0)
    tv1 = mg.random_test_vectors(P0.coarse_dims, 2 * nv[0], nv[1], 7002)
    Vc1, d1 = 2 * 2 * 2 * 4, 2 * nv[0]
    s.set_test_vectors(1, to_dev(tv1.reshape(nv[1], Vc1, d1).numpy()))
    s.setup(Ud, kappa_of(m0), 1.6, 0.003)
    P1 = mg.build_prolongation(tv1, agg[1], P0.coarse_dims, d1)
    Dc2 = mg.galerkin(Dc1, P1)
    return s, op, P0, Dc1, P1, Dc2, sap1


def test_second_coarsening_parity(injected_three_level):
    s, op, P0, Dc1, P1, Dc2, sap1 = injected_three_level
    say("3-level P / D_c parity")
    Vc2, d2 = s.level_info(2)
    D = torch.empty((Vc2, 9, d2, d2), dtype=torch.complex128, device=DEV)
    s.export(1, 2, D)
    D = D.cpu().transpose(-1, -2)
    assert rel(D[:, 0], Dc2.S.reshape(-1, d2, d2)) < 1e-12
    for m in range(4):
        assert rel(D[:, 1 + 2 * m], Dc2.F[m].reshape(-1, d2, d2)) < 1e-12
        assert rel(D[:, 2 + 2 * m], Dc2.B[m].reshape(-1, d2, d2)) < 1e-12


def test_coarse_sap_and_cycle(injected_three_level):
    s, op, P0, Dc1, P1, Dc2, sap1 = injected_three_level
    say("coarse SAP / level-1 cycle parity")
    Vc1, d1 = s.level_info(1)
    cd = P0.coarse_dims
    v = mg.random_test_vectors(cd, d1, 2, 7003)
    vd = to_dev(v.reshape(2, Vc1, d1).numpy())
    out = torch.empty_like(vd)
    mus = [0.003, -0.05]
    s.apply(tm.OP_SAP, 1, vd, out, mus)
    for r in range(2):
        ref = mg.sap(Dc1, v[r], torch.zeros_like(v[r]), mus[r], sap1, 2, 4)
        assert rel(out.cpu()[r], ref.reshape(Vc1, d1)) < 1e-11
    s.apply(tm.OP_PREC, 1, vd, out, mus)
    p = mg.MGParams(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16),
                    sap_block=((4, 4, 4, 4), sap1), coarsest_maxiter=50)
    H = mg.Hierarchy(op, p, 0.003)
    lvl1 = mg.Level(Dc1, 1, P=P1, nxt=mg.Level(Dc2, 2))
    for r in range(2):
        ref = H.precondition(lvl1, v[r], mus[r])
        assert rel(out.cpu()[r], ref.reshape(Vc1, d1)) < 1e-9


def coarse_op_from_export(s, level, cdims):
    """The library's stored D_c of `level` (exact values of its storage
    precision) as an oracle CoarseOp."""
    Vc, d = s.level_info(level)
    D = torch.empty((Vc, 9, d, d), dtype=torch.complex128, device=DEV)
    s.export(1, level, D)
    D = D.cpu().transpose(-1, -2)
    lx, ly, lz, lt = cdims
    blk = lambda b: D[:, b].reshape(lt, lz, ly, lx, d, d).contiguous()
    return mg.CoarseOp(blk(0), torch.stack([blk(1 + 2 * m) for m in range(4)]),
                       torch.stack([blk(2 + 2 * m) for m in range(4)])), Vc, d


def check_coarsest(s, level, cdims, nrhs, mus, iters, tol_rel, seed):
    Dc, Vc, d = coarse_op_from_export(s, level, cdims)
    v = mg.random_test_vectors(cdims, d, nrhs, seed)
    vd = to_dev(v.reshape(nrhs, Vc, d).numpy())
    out = torch.empty_like(vd)
    s.apply(tm.OP_COARSEST, level, vd, out, mus)
    for r in range(nrhs):
        ref = mg.fgmres(lambda e: Dc.apply(e, mus[r]), v[r], 1e-30, iters, iters).x
        err = rel(out.cpu()[r], ref.reshape(Vc, d))
        say(f"  rhs {r} mu {mus[r]}: rel. difference {err:.2e}")
        assert err < tol_rel


# GMRES with a fixed iteration count (tolerance below reach) has a unique
# iterate, the minimiser over the Krylov space, so the GPU result is
# compared with the oracle's GMRES on the same stored D_c.  Covered: the
# one-site-per-workgroup kernel (one RHS, 16-bit storage), the shared-site
# cooperative kernel (two RHS, FP32 storage, FP64) and the generic path.
@pytest.mark.parametrize("precision,storage,nrhs", [
    ("mixed", "bf16", 1), ("mixed", "fp16", 1), ("mixed", "bf16", 2), ("mixed", "fp32", 1),
    ("mixed", "bf16", 4), ("fp64", "fp64", 1), ("fp64", "fp64", 2)])
def test_coarsest_gmres_two_level(c1, precision, storage, nrhs):
    w, m0, U, Ud, op = c1
    say("coarsest GMRES, 2 levels", precision, storage, nrhs)
    prec = tm.MIXED if precision == "mixed" else tm.FP64
    st = {"bf16": tm.STORE_BF16, "fp16": tm.STORE_FP16, "fp32": tm.STORE_FP32, "fp64": tm.STORE_FP64}[storage]
    s = make_solver(w, precision=prec, storage=st, coarsest_iters=20, coarsest_tol=1e-30)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    cdims = tuple(a // b for a, b in zip(w.dims, w.agg[0]))
    mus = [w.mu, -0.05, 0.2, 0.0][:nrhs]
    check_coarsest(s, 1, cdims, nrhs, mus, 20, 1e-10 if prec == tm.FP64 else 1e-3, 7100 + nrhs)


def test_coarsest_gmres_three_level():
    dims = (8, 8, 16, 16)
    say("coarsest GMRES, 3 levels", dims)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1236)
    agg = ((4, 4, 4, 4), (2, 2, 2, 2))
    p = tm.default_params(nlevels=3, agg=agg, nv=(12, 16), sap_block1=(1, 1, 2, 2), coarsest_iters=24,
                          coarsest_tol=1e-30, setup_iters=1, precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(m0), 1.6, 0.003)
    cdims = tuple(a // b // c for a, b, c in zip(dims, agg[0], agg[1]))
    check_coarsest(s, 2, cdims, 1, [0.003], 24, 1e-3, 7200)


# Graph mode: the intermediate-level solve of every fine cycle is captured
# once per right-hand-side count and replayed.  The replayed kernels are the
# eager ones in the same order with fixed-order reductions, so every solve
# must match the eager solver bit for bit: three single-RHS solves in a row
# (capture on the second use, replays after), a 3-RHS batch with signed
# per-RHS mu (a second graph), then single RHS again, with eager test-hook
# work and host synchronisation between the solves.
def test_graph_captured_cycle_matches_eager():
    dims = (8, 8, 16, 16)
    say("graph-captured level-1 solve vs eager", dims)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1238)
    op = WilsonClover(U, m0, 1.6)
    base = dict(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16), sap_block1=(1, 1, 2, 2), setup_iters=1,
                l2_iters=6, coarsest_iters=10, precision=tm.MIXED, storage=tm.STORE_BF16)
    solvers = []
    for g in (0, 1):
        s = tm.Solver(dims, tm.default_params(use_graph=g, **base))
        s.setup(Ud, kappa_of(m0), 1.6, 0.003)
        solvers.append(s)
    cases = [(5101, 1, None), (5102, 1, None), (5103, 1, None), (5104, 3, [0.003, -0.003, 0.02]), (5105, 1, None)]
    for seed, n, mus in cases:
        b, bd = spinors(dims, seed, n)
        xs, infos = [], []
        for s in solvers:
            x = torch.empty_like(bd)
            info = s.solve(bd, x, mus, tol=1e-10)
            assert info.status == 0
            xs.append(x)
            infos.append(info)
            y = torch.empty_like(bd)
            s.apply(tm.OP_D64, 0, x, y, mus)   # eager work between the solves
            torch.cuda.synchronize()
        say("seed", seed, "nrhs", n, "outer", infos[0].outer_iters, infos[1].outer_iters)
        assert infos[0].outer_iters == infos[1].outer_iters
        assert torch.equal(xs[0], xs[1])
        mu_list = mus or [0.003] * n
        for r in range(n):
            res = norm(field(b[r]) - op.apply(field(xs[1].cpu()[r]), mu_list[r])) / norm(field(b[r]))
            assert res <= 1e-10


# The batched coarse operator and level-1 SAP on the matrix cores: 16
# right-hand sides per workgroup, bf16 D_c, each FP32 vector entry split
# into two bf16 parts (kept to 2^-18 of its size), FP32 accumulation.
# Checked against the oracle's FP64 arithmetic on the same stored D_c,
# with 20 right-hand sides (one full group of 16 and a ragged one) and
# per-RHS signed mu; 4 right-hand sides take the vector-ALU kernels on the
# same data.  Bars from the arithmetic: the split keeps each input to
# 4e-6, sums of a few hundred FP32 products add 1e-6.
@pytest.fixture(scope="module")
def mixed_three_level_d48():
    dims = (8, 8, 16, 16)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1237)
    agg = ((4, 4, 4, 4), (2, 2, 2, 2))
    sap1 = (1, 1, 2, 2)
    p = tm.default_params(nlevels=3, agg=agg, nv=(24, 32), sap_block1=sap1, setup_iters=1, precision=tm.MIXED,
                          storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(m0), 1.6, 0.003)
    cd1 = tuple(a // b for a, b in zip(dims, agg[0]))
    cd2 = tuple(a // b for a, b in zip(cd1, agg[1]))
    return s, cd1, cd2, sap1


# variant None: the launcher's own rule; 0 / 1 forced through the variant
# table (vector ALU with 20 right-hand sides, matrix cores with one).
@pytest.mark.parametrize("level,nrhs,variant", [(1, 20, None), (2, 20, None), (1, 4, None), (2, 4, None),
                                                (1, 20, 0), (2, 20, 0), (1, 1, 1), (2, 1, 1)])
def test_coarse_operator_batched_mixed(mixed_three_level_d48, level, nrhs, variant):
    s, cd1, cd2, sap1 = mixed_three_level_d48
    cdims = cd1 if level == 1 else cd2
    Dc, Vc, d = coarse_op_from_export(s, level, cdims)
    say(f"batched D_c, level {level} (d = {d}), {nrhs} RHS, variant {variant}, mixed bf16")
    mus = [0.003 * (1 + r) * (-1) ** r for r in range(nrhs)]
    v = mg.random_test_vectors(cdims, d, nrhs, 7300 + level)
    vd = to_dev(v.reshape(nrhs, Vc, d).numpy())
    out = torch.empty_like(vd)
    try:
        if variant is not None:
            tm.tune_set(tm.TUNE_COARSE_APPLY, d, Vc, nrhs, variant)
        s.apply(tm.OP_DC, level, vd, out, mus)
    finally:
        tm.tune_clear()
    worst = worst_el = 0.0
    for r in range(nrhs):
        ref = Dc.apply(v[r], mus[r])
        worst = max(worst, rel(out.cpu()[r], ref.reshape(Vc, d)))
        worst_el = max(worst_el, maxabs_rel(out.cpu()[r], ref.reshape(Vc, d)))
    say(f"  worst rel. difference {worst:.2e}, elementwise {worst_el:.2e}")
    assert worst < 2e-5 and worst_el < 2e-5


@pytest.mark.parametrize("nrhs,variant", [(20, None), (4, None), (20, 0), (1, 1), (20, 2), (1, 2), (20, 3), (4, 3),
                                          (1, 3)])
def test_coarse_sap_batched_mixed(mixed_three_level_d48, nrhs, variant):
    s, cd1, cd2, sap1 = mixed_three_level_d48
    Dc, Vc, d = coarse_op_from_export(s, 1, cd1)
    say(f"batched level-1 SAP (d = {d}), {nrhs} RHS, variant {variant}, mixed bf16")
    mus = [0.003 * (1 + r) * (-1) ** r for r in range(nrhs)]
    v = mg.random_test_vectors(cd1, d, nrhs, 7310)
    vd = to_dev(v.reshape(nrhs, Vc, d).numpy())
    out = torch.empty_like(vd)
    try:
        if variant is not None:
            tm.tune_set(tm.TUNE_SAP1, d, Vc, nrhs, variant)
        s.apply(tm.OP_SAP, 1, vd, out, mus)
    finally:
        tm.tune_clear()
    worst = worst_el = 0.0
    for r in range(nrhs):
        ref = mg.sap(Dc, v[r], torch.zeros_like(v[r]), mus[r], sap1, 2, 4)
        worst = max(worst, rel(out.cpu()[r], ref.reshape(Vc, d)))
        worst_el = max(worst_el, maxabs_rel(out.cpu()[r], ref.reshape(Vc, d)))
    say(f"  worst rel. difference {worst:.2e}, elementwise {worst_el:.2e}")
    assert worst < 1e-4 and worst_el < 1e-4


@pytest.mark.parametrize("nrhs", [20, 4])
def test_coarse_transfers_batched_mixed(mixed_three_level_d48, nrhs):
    """Level 1 -> 2 restriction (20 RHS: the matrix-core kernel) and level
    2 -> 1 prolongation against the oracle's FP64 transfers with the
    library's own rounded level-1 P."""
    s, cd1, cd2, sap1 = mixed_three_level_d48
    Vc1, d1 = s.level_info(1)
    Vc2, d2 = s.level_info(2)
    nv1 = d2 // 2
    say(f"batched level-1 transfers (d = {d1} -> {d2}), {nrhs} RHS, mixed bf16")
    P1 = torch.empty((nv1, Vc1, d1), dtype=torch.complex128, device=DEV)
    s.export(0, 1, P1)
    lx, ly, lz, lt = cd1
    V1 = P1.cpu().reshape(nv1, lt, lz, ly, lx, d1)
    agg1 = tuple(a // b for a, b in zip(cd1, cd2))
    Q = mg.to_blocks(V1, agg1, True).movedim(0, -1).contiguous()
    Pr = mg.Prolongation(Q, agg1, cd1, d1)
    v = mg.random_test_vectors(cd1, d1, nrhs, 7320)
    vd = to_dev(v.reshape(nrhs, Vc1, d1).numpy())
    rc = torch.empty((nrhs, Vc2, d2), dtype=torch.complex128, device=DEV)
    s.apply(tm.OP_RESTRICT, 1, vd, rc)
    ref = torch.stack([Pr.restrict(v[r]).reshape(Vc2, d2) for r in range(nrhs)])
    err_r = rel(rc.cpu(), ref)
    back = torch.empty_like(vd)
    s.apply(tm.OP_PROLONG, 2, rc, back)
    refp = torch.stack([Pr.prolong(rc.cpu()[r].reshape(*cd2[::-1], d2)).reshape(Vc1, d1) for r in range(nrhs)])
    err_p = rel(back.cpu(), refp)
    say(f"  P^dag {err_r:.2e}, P {err_p:.2e}")
    assert err_r < 2e-5 and err_p < 2e-5


def test_autotune_table_and_tuned_solve(mixed_three_level_d48, tmp_path):
    """The autotuner times both variants of every family for 1 and 20
    right-hand sides on this hierarchy, keeps the faster and writes the
    table as JSON; a solve with the tuned table still meets 1e-10 against
    the oracle's operator."""
    import json
    s, cd1, cd2, sap1 = mixed_three_level_d48
    path = tmp_path / "tune.json"
    tm.tune_clear()
    try:
        s.autotune([1, 20], reps=2, json_path=str(path))
        doc = json.loads(path.read_text())
        say("tuned", json.dumps(doc["entries"]))
        assert doc["format"] == "tmamg-tune-1"
        fams = {e["family"] for e in doc["entries"]}
        assert {"coarse_apply", "sap1", "restrict0", "prolong0", "sap0"} <= fams
        names = ["coarse_apply", "sap1", "restrict0", "prolong0", "sap0"]
        assert any(e["family"] == "sap1" and len(e["ms"]) == 4 for e in doc["entries"])
        for e in doc["entries"]:
            times = {v: t for v, t in e["ms"]}
            assert e["variant"] in times and times[e["variant"]] == min(times.values())
            assert tm.tune_get(names.index(e["family"]), *e["shape"]) == e["variant"]
        dims = (8, 8, 16, 16)
        m0 = load_m0()["c4"]
        U, _ = links(dims, 0.3, 1237)
        op = WilsonClover(U, m0, 1.6)
        b, bd = spinors(dims, 5201, 1)
        x = torch.empty_like(bd)
        info = s.solve(bd, x, tol=1e-10)
        assert info.status == 0
        assert norm(field(b[0]) - op.apply(field(x.cpu()[0]), 0.003)) / norm(field(b[0])) <= 1e-10
    finally:
        tm.tune_clear()


def test_setup_update_along_link_random_walk():
    """Setup reuse along slowly changing links (the paper updates the setup
    with one iteration per inversion along the trajectory): after a full
    setup at U_0, three random-walk steps U_k = exp(0.05 i g.lambda/2) U_{k-1},
    each followed by one setup iteration on the kept test vectors and a
    solve.  Every solve meets 1e-10 in the oracle's operator at U_k, and the
    updated hierarchy needs about as many outer iterations as a fresh full
    setup at the same links."""
    from lattice_inputs import md_step_links
    dims = (8, 8, 16, 16)
    say("setup update along a random walk", dims)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1239)
    p = tm.default_params(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16), sap_block1=(1, 1, 2, 2),
                          setup_iters=2, l2_iters=6, coarsest_iters=10, precision=tm.MIXED,
                          storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(m0), 1.6, 0.003)
    b, bd = spinors(dims, 5301, 1)
    for k in range(1, 4):
        U = md_step_links(U, 0.05, 5310 + k)
        s.setup_update(to_dev(U), 1)
        x = torch.empty_like(bd)
        info = s.solve(bd, x, tol=1e-10)
        op = WilsonClover(torch.as_tensor(U), m0, 1.6)
        res = norm(field(b[0]) - op.apply(field(x.cpu()[0]), 0.003)) / norm(field(b[0]))
        say(f"  step {k}: outer {info.outer_iters}, residual {res:.2e}")
        assert info.status == 0 and res <= 1e-10
    fresh = tm.Solver(dims, p)
    fresh.setup(to_dev(U), kappa_of(m0), 1.6, 0.003)
    x = torch.empty_like(bd)
    info_f = fresh.solve(bd, x, tol=1e-10)
    say(f"  fresh setup at the last links: outer {info_f.outer_iters}")
    assert info.outer_iters <= 1.5 * info_f.outer_iters + 2


# ------------------------------------------------------------------ degenerate and failure cases
def test_free_field_solve_matches_closed_form():
    """Unit links (the clover term vanishes, D is diagonal in momentum space):
    the multigrid solve at mu = 0 and at mu = 0.05 against the oracle's FFT
    closed form, on 8^4 whose 4^4 aggregates give a 2^4 coarse lattice where
    the +mu and -mu neighbours of a coarse site coincide.  Bar: residual
    1e-10 times the condition number of the free operator at m0 = 0.1
    (|lambda| from 0.1 to 8.1) gives 1e-8."""
    from lattice_inputs import unit_links
    from oracle.dirac import free_field_solve
    dims = (8, 8, 8, 8)
    m0 = 0.1
    U = unit_links(dims)
    p = tm.default_params(nlevels=2, nv=(12, 0), precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    s.setup(to_dev(U), kappa_of(m0), 1.7, 0.05)
    b, bd = spinors(dims, 5401, 2)
    x = torch.empty_like(bd)
    mus = [0.0, 0.05]
    info = s.solve(bd, x, mus, tol=1e-10)
    assert info.status == 0
    for r in range(2):
        ref = free_field_solve(field(b[r]), m0, mus[r])
        err = rel(field(x.cpu()[r]), ref)
        say(f"  free field, mu = {mus[r]}: {err:.2e}")
        assert err < 1e-8


def test_zero_and_mixed_right_hand_sides(c1):
    """A zero right-hand side is solved by x = 0 at once; in a batch with a
    nonzero one it stays exactly zero while the other converges."""
    w, m0, U, Ud, op = c1
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_BF16)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, 5402, 2)
    bd[0].zero_()
    x = torch.full_like(bd, 7.0)
    info = s.solve(bd, x, tol=1e-10)
    assert info.status == 0
    assert torch.count_nonzero(x[0]) == 0
    assert norm(field(b[1]) - op.apply(field(x.cpu()[1]), w.mu)) / norm(field(b[1])) <= 1e-10
    z = torch.zeros_like(bd[:1])
    x1 = torch.full_like(z, 3.0)
    info = s.solve(z, x1, tol=1e-10)
    assert info.status == 0 and info.outer_iters == 0 and torch.count_nonzero(x1) == 0


def test_failure_paths_report_status(c1):
    """Non-unitary links and NaN right-hand sides are refused with
    TMAMG_ENUMERIC before any iteration; a solve before setup is a state
    error; the context stays usable afterwards."""
    w, m0, U, Ud, op = c1
    s = make_solver(w, precision=tm.MIXED, storage=tm.STORE_BF16)
    b, bd = spinors(w.dims, 5403, 1)
    x = torch.empty_like(bd)
    with pytest.raises(tm.TmamgError) as e:
        s.solve(bd, x)
    assert e.value.status == tm.binding.ESTATE
    with pytest.raises(tm.TmamgError) as e:
        s.setup(Ud * 1.01, kappa_of(m0), w.csw, w.mu)
    assert e.value.status == tm.binding.ENUMERIC
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    bad = bd.clone()
    bad[0, 1, 2, 3, 4, 0, 0] = float("nan")
    with pytest.raises(tm.TmamgError) as e:
        s.solve(bad, x)
    assert e.value.status == tm.binding.ENUMERIC
    info = s.solve(bd, x, tol=1e-10)
    assert info.status == 0
    assert norm(field(b[0]) - op.apply(field(x.cpu()[0]), w.mu)) / norm(field(b[0])) <= 1e-10
