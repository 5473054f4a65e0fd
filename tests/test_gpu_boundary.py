"""The C ABI's conventions on the GPU: internal buffers from the caller's
allocator (torch's caching allocator), the ordering of the library's stream
against the caller's, the D^dag operator hook, solves from an initial
guess, the per-level iteration totals in tmamg_info, and the failure path
of the persistent coarse kernels' bounded barrier wait."""
import pytest
import torch

from lattice_inputs import workload, load_m0
from oracle.dirac import WilsonClover, norm
from tests.gpu_common import DEV, links, spinors, kappa_of, rel, field

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c1():
    w = workload("c1")
    m0 = load_m0()["c1"]
    U, Ud = links(w.dims, w.eps, w.seeds["links"])
    return w, m0, U, Ud, WilsonClover(U, m0, w.csw)


def params(w, **kw):
    p = dict(nlevels=2, agg=w.agg, nv=w.nv, setup_iters=w.setup_iters, init_smooth=w.init_smooth,
             sap_sweeps=w.sap_sweeps, mr_steps=w.mr_steps, restart=w.restart)
    p.update(kw)
    return tm.default_params(**p)


def three_level_params(**kw):
    p = dict(nlevels=3, agg=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16), sap_block1=(1, 1, 2, 2),
             setup_iters=1, init_smooth=2, coarsest_iters=20, l2_iters=4, restart=20)
    p.update(kw)
    return tm.default_params(**p)


def test_internal_buffers_come_from_torch_allocator(c1):
    """With the default allocator the hierarchy is torch memory: it shows up
    in torch.cuda.memory_allocated and goes back on close; with hipMalloc
    (allocator=None) torch sees none of it.  Both solve to the same bits."""
    w, m0, U, Ud, op = c1
    say("allocator: torch vs hipMalloc")
    b, bd = spinors(w.dims, 8801, 1)
    x1, x2 = torch.empty_like(bd), torch.empty_like(bd)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    s = tm.Solver(w.dims, params(w, precision=tm.MIXED))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    i1 = s.solve(bd, x1, tol=1e-10)
    held = torch.cuda.memory_allocated() - base
    say(f"  torch-allocated by the context: {held / 2**20:.1f} MiB")
    # links (FP64 + FP32), clover, test vectors, P, D_c and the Krylov bases
    assert held > 4096 * (4 * 9 * 24 + 72 * 12 + 24 * 12 * 12)
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    s2 = tm.Solver(w.dims, params(w, precision=tm.MIXED), allocator=None)
    s2.setup(Ud, kappa_of(m0), w.csw, w.mu)
    assert torch.cuda.memory_allocated() == base
    i2 = s2.solve(bd, x2, tol=1e-10)
    s2.close()
    assert i1.status == 0 and i2.status == 0 and i1.outer_iters == i2.outer_iters
    assert torch.equal(x1, x2)


def test_ddag_operator(c1):
    w, m0, U, Ud, op = c1
    say("D^dag hook, FP64 and FP32")
    s = tm.Solver(w.dims, params(w, nlevels=0, setup_iters=0, init_smooth=0, precision=tm.MIXED,
                                 storage=tm.STORE_FP32))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    psi, psid = spinors(w.dims, 8802, 2)
    mus = [w.mu, -0.07]
    out = torch.empty_like(psid)
    ref = torch.stack([op.apply_dag(field(psi[r]), mus[r]) for r in range(2)])
    s.apply(tm.OP_DDAG64, 0, psid, out, mus)
    assert rel(field(out.cpu()), ref) < 1e-13
    s.apply(tm.OP_DDAG32, 0, psid, out, mus)
    assert rel(field(out.cpu()), ref) < 2e-6
    # <D^dag psi, chi> = <psi, D chi>
    chi = torch.as_tensor(spinors(w.dims, 8803, 1)[0][0])
    lhs = torch.vdot(ref[0].reshape(-1), field(chi).reshape(-1))
    rhs = torch.vdot(field(torch.as_tensor(psi[0])).reshape(-1), op.apply(field(chi), mus[0]).reshape(-1))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    s.close()


def test_inputs_written_on_the_callers_stream(c1):
    """The library runs on its own stream.  A right-hand side written on the
    caller's current stream just before the call, with that stream still
    busy, is complete when the library reads it, and the solution is
    complete before the caller's next work on its stream reads it."""
    w, m0, U, Ud, op = c1
    say("stream ordering: input and output on a busy caller stream")
    s = tm.Solver(w.dims, params(w, precision=tm.MIXED), stream=torch.cuda.Stream(device=DEV))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, 8811, 1)
    filler = torch.ones(1 << 26, device=DEV)
    torch.cuda.synchronize()
    caller = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(caller):
        for _ in range(8):
            filler.mul_(1.0000001)   # 256 MiB of work ahead of the input
        b2 = bd * 2.0
        x = torch.empty_like(bd)
        s.solve(b2, x, tol=1e-10)
        y = x * 0.5
    torch.cuda.synchronize()
    res = op.apply(field(y.cpu()[0]), w.mu) - field(torch.as_tensor(b[0]))
    assert norm(res) / norm(field(torch.as_tensor(b[0]))) < 1e-9
    s.close()


def test_solve_from_initial_guess(c1):
    """A solution as the guess needs no iteration; a perturbed one
    converges to the oracle-checked residual; a guess worse than zero is
    replaced by zero (the same iterations as a cold start)."""
    w, m0, U, Ud, op = c1
    say("solve from an initial guess")
    s = tm.Solver(w.dims, params(w, precision=tm.MIXED))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, 8804, 2)
    x = torch.empty_like(bd)
    cold = s.solve(bd, x, tol=1e-12)
    assert cold.status == 0
    x0 = x.clone()
    warm = s.solve(bd, x0, tol=1e-10, guess=True)
    assert warm.status == 0 and warm.outer_iters == 0
    xp = x + 1e-4 * torch.randn(x.shape, dtype=torch.complex128, device=DEV)
    near = s.solve(bd, xp, tol=1e-10, guess=True)
    say(f"  cold {cold.outer_iters} (to 1e-12), perturbed guess {near.outer_iters} (to 1e-10)")
    assert near.status == 0 and 0 < near.outer_iters
    for r in range(2):
        assert norm(field(b[r]) - op.apply(field(xp.cpu()[r]), w.mu)) / norm(field(b[r])) <= 1e-10
    bad = 1e3 * torch.randn(x.shape, dtype=torch.complex128, device=DEV)
    c2 = s.solve(bd, torch.empty_like(bd), tol=1e-10)
    wild = s.solve(bd, bad, tol=1e-10, guess=True)
    assert wild.status == 0 and wild.outer_iters == c2.outer_iters
    s.close()


def test_info_counts_coarse_iterations():
    """Three levels: the intermediate FGMRES steps and the coarsest GMRES
    iterations of a solve are reported, and grow with the batch."""
    dims = (8, 8, 8, 16)
    say("info: per-level iteration totals")
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1235)
    s = tm.Solver(dims, three_level_params(precision=tm.MIXED))
    s.setup(Ud, kappa_of(m0), 1.6, 0.01)
    b, bd = spinors(dims, 8805, 2)
    x = torch.empty_like(bd)
    info = s.solve(bd, x, tol=1e-10)
    say(f"  {info.as_dict()}")
    assert info.status == 0
    assert info.l2_iters_total >= info.outer_iters
    assert info.coarsest_iters_total >= info.l2_iters_total
    one = s.solve(bd[:1].contiguous(), x[:1].contiguous(), tol=1e-10)
    assert 0 < one.coarsest_iters_total <= info.coarsest_iters_total
    s.close()


def test_barrier_timeout_becomes_a_status():
    """A persistent coarse kernel whose bounded barrier wait gave up makes
    the solve return TMAMG_EHIP (the timeout is marked from the host; no
    kernel is made to wait); the context then uses the generic coarse
    kernels and solves normally, to the same residual."""
    dims = (8, 8, 8, 16)
    say("barrier timeout -> status")
    m0 = load_m0()["c4"]
    U, Ud = links(dims, 0.3, 1235)
    op = WilsonClover(U, m0, 1.6)
    s = tm.Solver(dims, three_level_params(precision=tm.MIXED))
    s.setup(Ud, kappa_of(m0), 1.6, 0.01)
    b, bd = spinors(dims, 8806, 1)
    x = torch.empty_like(bd)
    ok = s.solve(bd, x, tol=1e-10)
    assert ok.status == 0
    s.inject_barrier_timeout()
    with pytest.raises(tm.TmamgError) as e:
        s.solve(bd, x, tol=1e-10)
    assert e.value.status == tm.binding.EHIP and "barrier" in str(e.value)
    again = s.solve(bd, x, tol=1e-10)
    say(f"  after the fallback: {again.as_dict()}")
    assert again.status == 0
    assert norm(field(b[0]) - op.apply(field(x.cpu()[0]), 0.01)) / norm(field(b[0])) <= 1e-10
    s.close()


@pytest.mark.parametrize("levels", [2, 3])
def test_setup_memory_plan(c1, levels):
    """The memory plan: the setup treating the test vectors in chunks of 5
    (12 and 16 vectors: chunks of 5, 5, 2 and 5, 5, 5, 1) and releasing them
    afterwards gives the hierarchy of the all-at-once setup (FP64: the same
    vectors up to the rounding of differently batched coarse solves), solves
    to the same tolerance in the same number of outer iterations, and
    refuses setup updates once the test vectors are gone."""
    w, m0, U, Ud, op = c1
    say("memory plan,", levels, "levels")
    mk = (lambda **kw: params(w, **kw)) if levels == 2 else three_level_params
    ref = tm.Solver(w.dims, mk())
    ref.setup(Ud, kappa_of(m0), w.csw, w.mu)
    s = tm.Solver(w.dims, mk(setup_chunk=5, keep_test_vectors=0))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    for what, level in ((0, 0), (1, 1)):
        a = torch.empty(ref.params.nv[0] * ref.volume * 12 if what == 0 else
                        ref.level_info(1)[0] * 9 * ref.level_info(1)[1] ** 2, dtype=torch.complex128, device=DEV)
        b = torch.empty_like(a)
        ref.export(what, level, a)
        s.export(what, level, b)
        d = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a))
        say(f"  {'P' if what == 0 else 'D_c'} level {level}: rel. difference {d:.2e}")
        assert d < 1e-8
    psi, psid = spinors(w.dims, 4401, 1)
    xr, xs = torch.empty_like(psid), torch.empty_like(psid)
    ir = ref.solve(psid, xr, tol=1e-10)
    i_s = s.solve(psid, xs, tol=1e-10)
    res = norm(field(psi[0]) - op.apply(field(xs.cpu()[0]), w.mu)) / norm(field(psi[0]))
    say(f"  outer iterations {ir.outer_iters} / {i_s.outer_iters}; oracle residual {res:.2e}")
    assert i_s.status == 0 and res <= 1e-10 and abs(i_s.outer_iters - ir.outer_iters) <= 1
    with pytest.raises(tm.TmamgError) as e:
        s.setup_update(Ud, 1)
    assert e.value.status == -5   # TMAMG_ESTATE
    ref.setup_update(Ud, 1)
    ref.close()
    s.close()
