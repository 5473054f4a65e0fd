"""GPU parity of the non-degenerate doublet solve (Sec. 1.1, Eq. 2) through
the C ABI: the FP64 true residual of D_ND(mubar, epsbar) x = b recomputed by
the oracle's doublet operator, the unit-link solve against the oracle's
momentum-space closed form, and the decoupled case against two light-sector
solves."""
import sys

import pytest
import torch

from lattice_inputs import workload, load_m0, unit_links
from oracle.dirac import WilsonClover, norm
from oracle.nd import NDOperator, free_field_nd_solve, coarse_nd_apply, sap_doublet
from oracle import mg
from tests.gpu_common import links, spinors, kappa_of, rel, field, to_dev

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c1():
    w = workload("c1")
    m0 = load_m0()["c1"]
    U, Ud = links(w.dims, w.eps, w.seeds["links"])
    return w, m0, U, Ud, WilsonClover(U, m0, w.csw)


def solver(w, precision, nlevels=2):
    p = dict(nlevels=nlevels, agg=w.agg, nv=w.nv, setup_iters=w.setup_iters, init_smooth=w.init_smooth,
             sap_sweeps=w.sap_sweeps, mr_steps=w.mr_steps, restart=w.restart, precision=precision)
    if precision == tm.MIXED:
        p["storage"] = tm.STORE_BF16
    return tm.Solver(w.dims, tm.default_params(**p))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("mubar,epsbar", [(0.12, 0.10), (0.15, 0.05), (0.05, 0.12)])
def test_doublet_solve_true_residual(c1, precision, mubar, epsbar):
    """Bar: ||b - D_ND x|| / ||b|| <= 1e-10 with D_ND the oracle's (FP64)."""
    w, m0, U, Ud, op = c1
    say(f"doublet solve c1 {precision} mubar={mubar} epsbar={epsbar}")
    s = solver(w, tm.FP64 if precision == "fp64" else tm.MIXED)
    s.setup(Ud, kappa_of(m0), w.csw, mubar)
    b, bd = spinors(w.dims, 6101, 2)
    x = torch.empty_like(bd)
    info = s.solve_nd(bd, x, mubar, epsbar, tol=1e-10)
    assert info.status == 0
    nd = NDOperator(op, mubar, epsbar)
    bf = field(b)
    res = norm(bf - nd.apply(field(x.cpu()))) / norm(bf)
    say(f"  {info.outer_iters} outer iterations, oracle residual {res:.2e} (library {info.true_rel_resid:.2e})")
    assert res <= 1e-10
    assert abs(res - info.true_rel_resid) <= 1e-12


def test_doublet_unit_links_matches_closed_form():
    """Unit links: the doublet solve against the oracle's FFT solve with one
    8 x 8 spin-flavour matrix per momentum.  Bar 1e-8: the residual bound
    1e-10 times the condition number of the free doublet at m0 = 0.1."""
    dims = (8, 8, 8, 8)
    m0, mubar, epsbar = 0.1, 0.06, 0.04
    p = tm.default_params(nlevels=2, nv=(12, 0), precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    s.setup(to_dev(unit_links(dims)), kappa_of(m0), 1.7, mubar)
    b, bd = spinors(dims, 6102, 2)
    x = torch.empty_like(bd)
    info = s.solve_nd(bd, x, mubar, epsbar, tol=1e-10)
    assert info.status == 0
    err = rel(field(x.cpu()), free_field_nd_solve(field(b), m0, mubar, epsbar))
    say(f"  free doublet: {err:.2e} after {info.outer_iters} outer iterations")
    assert err < 1e-8


def test_decoupled_doublet_equals_light_solves(c1):
    """epsbar = 0: the doublet splits into D(mubar) x_0 = b_0 and
    D(-mubar) x_1 = b_1; both routes meet the 1e-10 residual, so their
    solutions agree to the condition number times 1e-10 (bar 1e-7)."""
    w, m0, U, Ud, op = c1
    mubar = 0.08
    s = solver(w, tm.MIXED)
    s.setup(Ud, kappa_of(m0), w.csw, mubar)
    b, bd = spinors(w.dims, 6103, 2)
    x = torch.empty_like(bd)
    assert s.solve_nd(bd, x, mubar, 0.0, tol=1e-10).status == 0
    y = torch.empty_like(bd)
    assert s.solve(bd, y, [mubar, -mubar], tol=1e-10).status == 0
    err = rel(x.cpu(), y.cpu())
    say(f"  decoupled doublet vs two solves: {err:.2e}")
    assert err < 1e-7


def test_doublet_argument_errors(c1):
    w, m0, U, Ud, op = c1
    s = solver(w, tm.MIXED)
    b, bd = spinors(w.dims, 6104, 2)
    x = torch.empty_like(bd)
    with pytest.raises(tm.TmamgError):
        s.solve_nd(bd, x, 0.1, 0.1)          # before setup
    s.setup(Ud, kappa_of(m0), w.csw, 0.1)
    with pytest.raises(ValueError):
        s.solve_nd(bd[:1], x[:1], 0.1, 0.1)  # one flavour
    with pytest.raises(tm.TmamgError):
        s.solve_nd(bd, x, float("nan"), 0.1)


def test_doublet_three_level_mixed():
    """Three levels (4^4 then 2^4 aggregates, the bench's shape of hierarchy)
    on 8^3x16: the two flavours' coarsest solves run as one launch each.
    Bar: the oracle's doublet residual <= 1e-10."""
    dims = (8, 8, 8, 16)
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1235)
    op = WilsonClover(U, m0, 1.6)
    p = tm.default_params(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16), sap_block1=(2, 2, 2, 2),
                          precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    mubar, epsbar = 0.13, 0.11
    s.setup(Ud, kappa_of(m0), 1.6, 0.01)
    b, bd = spinors(dims, 6105, 2)
    x = torch.empty_like(bd)
    info = s.solve_nd(bd, x, mubar, epsbar, tol=1e-10)
    assert info.status == 0
    bf = field(b)
    res = norm(bf - NDOperator(op, mubar, epsbar).apply(field(x.cpu()))) / norm(bf)
    say(f"  three-level doublet: {info.outer_iters} outer iterations, oracle residual {res:.2e}")
    assert res <= 1e-10


def test_doublet_graph_replay_matches_eager():
    """Intermediate-level solves replayed from captured HIP graphs (two
    flavours, so two coarsest launches per capture) give the same bits and
    iteration counts as plain launches, over three doublet solves in a row
    with eager work between them."""
    dims = (8, 8, 16, 16)
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
    for seed, (mubar, epsbar) in ((6201, (0.13, 0.11)), (6202, (0.13, 0.11)), (6203, (0.2, 0.05))):
        b, bd = spinors(dims, seed, 2)
        xs, iters = [], []
        for s in solvers:
            x = torch.empty_like(bd)
            info = s.solve_nd(bd, x, mubar, epsbar, tol=1e-10)
            assert info.status == 0
            xs.append(x)
            iters.append(info.outer_iters)
            y = torch.empty_like(bd)
            s.apply(tm.OP_D64, 0, x, y, [mubar, -mubar])   # eager work between the solves
            torch.cuda.synchronize()
        say(f"  doublet graph replay seed {seed}: outer {iters}")
        assert iters[0] == iters[1]
        assert torch.equal(xs[0], xs[1])
        bf = field(b)
        res = norm(bf - NDOperator(op, mubar, epsbar).apply(field(xs[1].cpu()))) / norm(bf)
        assert res <= 1e-10


@pytest.mark.parametrize("mubar,epsbar", [(0.12, 0.10), (0.05, 0.12)])
def test_doublet_coarse_operator_is_galerkin_product(c1, mubar, epsbar):
    """The library's doublet coarse operator (FP64 hierarchy, level 1)
    against the oracle's P_ND^dag D_ND P_ND with the library's own P:
    prolong each flavour, apply D_ND, restrict (Sec. 1.1 after Eq. 2)."""
    w, m0, U, Ud, op = c1
    say(f"D_ND,c parity c1 mubar={mubar} epsbar={epsbar}")
    s = solver(w, tm.FP64)
    s.setup(Ud, kappa_of(m0), w.csw, mubar)
    nv = w.nv[0]
    lx, ly, lz, lt = w.dims
    Pg = torch.empty((nv, lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device="cuda:0")
    s.export(0, 0, Pg)
    Q = mg.to_blocks(field(Pg.cpu()), w.agg[0], True).movedim(0, -1).contiguous()
    P = mg.Prolongation(Q, w.agg[0], w.dims, 12)
    Vc, d = s.level_info(1)
    e = mg.random_test_vectors(P.coarse_dims, d, 2, 6601)
    out = torch.empty((2, Vc, d), dtype=torch.complex128, device="cuda:0")
    s.apply(tm.OP_DCND, 1, to_dev(e.reshape(2, Vc, d).numpy()), out, [mubar, epsbar])
    ref = coarse_nd_apply(op, P, mubar, epsbar, e).reshape(2, Vc, d)
    err = rel(out.cpu(), ref)
    say(f"  rel. difference {err:.2e}")
    assert err < 1e-12
    s.close()


@pytest.mark.parametrize("mubar,epsbar", [(0.12, 0.10), (0.05, 0.12)])
def test_doublet_coupled_coarse_levels_converge_faster(mubar, epsbar):
    """Three levels on 8^3 x 16: the doublet solve with the coarse levels
    on D_ND,c (default) and with each flavour's own coarse cycle; both meet
    the oracle's residual bar, the coupled one in fewer outer iterations."""
    dims = (8, 8, 8, 16)
    w = workload("c4")
    m0 = load_m0()["c4"]
    U, Ud = links(dims, w.eps, 6701)
    op = WilsonClover(U, m0, w.csw)
    b, bd = spinors(dims, 6702, 2)
    its = {}
    for coupled in (1, 0):
        p = tm.default_params(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(24, 32), sap_block1=(2, 2, 2, 2),
                              setup_iters=3, init_smooth=2, coarsest_iters=10, l2_iters=6, restart=30,
                              precision=tm.MIXED, storage=tm.STORE_BF16, nd_coarse_coupling=coupled)
        s = tm.Solver(dims, p)
        s.setup(Ud, kappa_of(m0), w.csw, mubar)
        x = torch.empty_like(bd)
        info = s.solve_nd(bd, x, mubar, epsbar, tol=1e-10)
        nd = NDOperator(op, mubar, epsbar)
        res = norm(field(b) - nd.apply(field(x.cpu()))) / norm(field(b))
        say(f"  coupled coarse levels {coupled}: {info.outer_iters} outer iterations, oracle residual {res:.2e}")
        assert info.status == 0 and res <= 1e-10
        its[coupled] = info.outer_iters
        s.close()
    assert its[1] <= its[0]


def test_doublet_sap_on_coupled_blocks(c1):
    """The mixed-precision doublet SAP (the two flavours in one workgroup,
    the block operator with the flavour coupling -epsbar, one MR alpha per
    block over both flavours) against the oracle's coupled SAP in FP64 at
    the same sweeps and MR steps.  Bar as for the light-sector FP32 SAP."""
    w, m0, U, Ud, op = c1
    mubar, epsbar = 0.05, 0.12
    say(f"doublet SAP c1 mubar={mubar} epsbar={epsbar}")
    s = solver(w, tm.MIXED)
    s.setup(Ud, kappa_of(m0), w.csw, mubar)
    b, bd = spinors(w.dims, 6801, 2)
    out = torch.empty_like(bd)
    s.apply(tm.OP_SAPND, 0, bd, out, [mubar, epsbar])
    ref = sap_doublet(NDOperator(op, mubar, epsbar), field(b), w.sap_block[0], w.sap_sweeps[0], w.mr_steps)
    err = rel(field(out.cpu()), ref)
    say(f"  rel. difference {err:.2e}")
    assert err < 1e-5
    s.close()
