"""Components at the shapes the 24^3 x 48 bench hierarchy runs them, on
the library's own stored D_c (exported exactly), against the oracle:

* the coarsest GMRES on the 3^3 x 6 level (162 sites, 64 dof per site: the
  one-site-per-workgroup persistent kernel) at a fixed step count, one and
  two right-hand sides, against the oracle's GMRES run for the same steps;
* the level-1 SAP on the 6^3 x 12 level with 3^4 blocks (2 sweeps of 4 MR
  steps; one right-hand side on the vector ALU, eight on the matrix cores in
  each of their variants) against the oracle's SAP;
* the level-1 SAP of the 32^3 x 64 batched hierarchy (8^3 x 16 level, 2^4
  blocks) at its 12 right-hand sides, where one workgroup per SAP block runs
  the colour in one launch, two of the right-hand sides against the
  oracle's SAP.

A wrong coarse component only costs outer iterations in a full solve (the
FP64 residual still reaches 1e-10), so these shapes need checks of their own.
Bars: FP32 arithmetic on bf16-exact operators over 10 GMRES steps or 16 MR
steps, l2 and elementwise against the largest entry."""
import pytest
import torch

from lattice_inputs import workload, gauge_links, load_m0
from oracle import mg
from tests.gpu_common import DEV, to_dev, kappa_of, rel, maxabs_rel
from tests.test_gpu_parity import coarse_op_from_export

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c2_hierarchy():
    import bench
    w = workload("c2")
    m0 = load_m0()[w.name]
    say("c2 bench hierarchy: inputs", w.dims)
    Ud = to_dev(gauge_links(w.dims, w.eps, w.seeds["links"]))
    p = bench.solver_params(tm, w, tm.MIXED)
    p.coarsest_tol = 1e-12   # the coarsest GMRES runs all of its steps
    s = tm.Solver(w.dims, p)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    cd1 = tuple(w.dims[m] // w.agg[0][m] for m in range(4))
    cd2 = tuple(cd1[m] // w.agg[1][m] for m in range(4))
    yield w, s, cd1, cd2, p.coarsest_iters
    s.close()


@pytest.mark.parametrize("nrhs", [1, 2])
def test_coarsest_gmres_bench_shape(c2_hierarchy, nrhs):
    w, s, cd1, cd2, iters = c2_hierarchy
    Dc, Vc, d = coarse_op_from_export(s, 2, cd2)
    assert (Vc, d) == (162, 64)
    say(f"coarsest GMRES, {Vc} sites x {d} dof, {iters} steps, {nrhs} RHS")
    mus = [w.mu, -0.02][:nrhs]
    v = mg.random_test_vectors(cd2, d, nrhs, 9100 + nrhs)
    vd = to_dev(v.reshape(nrhs, Vc, d).numpy())
    out = torch.empty_like(vd)
    s.apply(tm.OP_COARSEST, 2, vd, out, mus)
    for r in range(nrhs):
        ref = mg.fgmres(lambda e: Dc.apply(e, mus[r]), v[r], 1e-30, iters, iters)
        assert ref.iters == iters
        got = out.cpu()[r]
        e2, ee = rel(got, ref.x.reshape(Vc, d)), maxabs_rel(got, ref.x.reshape(Vc, d))
        say(f"  rhs {r}: l2 {e2:.2e}, elementwise {ee:.2e} (oracle implicit residual {ref.resid[-1]:.2e})")
        assert e2 < 1e-4 and ee < 1e-4


@pytest.mark.parametrize("nrhs,variant", [(1, None), (8, 0), (8, 1), (8, 2)])
def test_level1_sap_bench_shape(c2_hierarchy, nrhs, variant):
    w, s, cd1, cd2, iters = c2_hierarchy
    Dc, Vc, d = coarse_op_from_export(s, 1, cd1)
    assert (Vc, d) == (2592, 48) and tuple(w.sap_block[1]) == (3, 3, 3, 3)
    say(f"level-1 SAP, {Vc} sites x {d} dof, blocks {w.sap_block[1]}, {nrhs} RHS, variant {variant}")
    mus = [0.0015 * (1 + r) * (-1) ** r for r in range(nrhs)]
    v = mg.random_test_vectors(cd1, d, nrhs, 9200 + nrhs)
    vd = to_dev(v.reshape(nrhs, Vc, d).numpy())
    out = torch.empty_like(vd)
    try:
        if variant is not None:
            tm.tune_set(tm.TUNE_SAP1, d, Vc, nrhs, variant)
        s.apply(tm.OP_SAP, 1, vd, out, mus)
    finally:
        if variant is not None:
            tm.tune_set(tm.TUNE_SAP1, d, Vc, nrhs, -1)
    worst = worst_el = 0.0
    for r in range(nrhs):
        ref = mg.sap(Dc, v[r], torch.zeros_like(v[r]), mus[r], w.sap_block[1], w.sap_sweeps[1], w.mr_steps)
        worst = max(worst, rel(out.cpu()[r], ref.reshape(Vc, d)))
        worst_el = max(worst_el, maxabs_rel(out.cpu()[r], ref.reshape(Vc, d)))
    say(f"  worst l2 {worst:.2e}, elementwise {worst_el:.2e}")
    assert worst < 1e-4 and worst_el < 1e-4


@pytest.fixture(scope="module")
def c3_hierarchy():
    import bench
    w = workload("c3")
    m0 = load_m0()[w.name]
    say("c3 bench hierarchy: inputs", w.dims)
    Ud = to_dev(gauge_links(w.dims, w.eps, w.seeds["links"], workers=8))
    s = tm.Solver(w.dims, bench.solver_params(tm, w, tm.MIXED))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    del Ud
    cd1 = tuple(w.dims[m] // w.agg[0][m] for m in range(4))
    yield w, s, cd1
    s.close()


def test_level1_sap_block_kernel_bench_shape(c3_hierarchy):
    w, s, cd1 = c3_hierarchy
    Dc, Vc, d = coarse_op_from_export(s, 1, cd1)
    assert (Vc, d) == (8192, 48) and tuple(w.sap_block[1]) == (2, 2, 2, 2)
    nrhs = w.extra["n_point"]
    say(f"level-1 SAP, {Vc} sites x {d} dof, blocks {w.sap_block[1]}, {nrhs} RHS (one workgroup per block)")
    mus = [0.0015 * (1 + r) * (-1) ** r for r in range(nrhs)]
    v = mg.random_test_vectors(cd1, d, nrhs, 9300)
    vd = to_dev(v.reshape(nrhs, Vc, d).numpy())
    out = torch.empty_like(vd)
    s.apply(tm.OP_SAP, 1, vd, out, mus)
    worst = worst_el = 0.0
    for r in (0, 7):
        ref = mg.sap(Dc, v[r], torch.zeros_like(v[r]), mus[r], w.sap_block[1], w.sap_sweeps[1], w.mr_steps)
        worst = max(worst, rel(out.cpu()[r], ref.reshape(Vc, d)))
        worst_el = max(worst_el, maxabs_rel(out.cpu()[r], ref.reshape(Vc, d)))
    say(f"  worst l2 {worst:.2e}, elementwise {worst_el:.2e}")
    assert worst < 1e-4 and worst_el < 1e-4
