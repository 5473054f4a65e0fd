"""The 24^3 x 48 workload at its full size, in the configuration the bench
times, against the oracle on the CPU: the fine stencil (FP64 and FP32) on
the whole lattice, and the mixed-precision three-level solve checked by the
property that defines its result, the true relative residual
||b - D x|| / ||b|| <= 1e-10 computed with the oracle's own FP64 operator.
Each test takes of the order of a minute, mostly for the oracle's clover
build and the input generation on the host."""
import os
import sys

import pytest
import torch

from lattice_inputs import workload, gauge_links, gaussian_spinor, load_m0
from oracle.dirac import WilsonClover, norm
from tests.gpu_common import DEV, to_dev, kappa_of, rel, field

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c2_full():
    w = workload("c2")
    m0 = load_m0()[w.name]
    say("c2 full size: inputs", w.dims)
    U = gauge_links(w.dims, w.eps, w.seeds["links"])
    Ud = to_dev(U)
    op = WilsonClover(torch.as_tensor(U), m0, w.csw)
    b = gaussian_spinor(w.dims, w.seeds["source"], n=1)
    return w, m0, Ud, op, b


def test_stencil_full_lattice(c2_full):
    w, m0, Ud, op, b = c2_full
    say("c2 stencil, whole lattice")
    p = tm.default_params(nlevels=w.nlevels, agg=w.agg, nv=w.nv, sap_block1=w.sap_block[1], setup_iters=0,
                          init_smooth=0, precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(w.dims, p)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    bd = to_dev(b)
    out = torch.empty_like(bd)
    ref = op.apply(field(b[0]), w.mu)
    s.apply(tm.OP_D64, 0, bd, out, [w.mu])
    e64 = rel(field(out.cpu()[0]), ref)
    s.apply(tm.OP_D32, 0, bd, out, [w.mu])
    e32 = rel(field(out.cpu()[0]), ref)
    say(f"  FP64 {e64:.2e}, FP32 {e32:.2e}")
    s.close()
    assert e64 < 1e-13 and e32 < 2e-6


def test_solve_full_size_bench_configuration(c2_full):
    import bench
    w, m0, Ud, op, b = c2_full
    say("c2 mixed three-level solve, bench configuration")
    s = tm.Solver(w.dims, bench.solver_params(tm, w, tm.MIXED))
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    bd = to_dev(b)
    x = torch.empty_like(bd)
    info = s.solve(bd, x, tol=w.tol)
    say("  info", info.as_dict())
    s.close()
    bf = field(b[0])
    res = norm(bf - op.apply(field(x.cpu()[0]), w.mu)) / norm(bf)
    say(f"  true relative residual (oracle operator, FP64) {res:.2e}")
    assert info.status == 0
    assert res <= 1e-10


def random_su3_directions(shape, seed):
    """Traceless anti-Hermitian 3x3 per link: a direction of U -> exp(tX) U."""
    g = torch.Generator().manual_seed(seed)
    A = torch.complex(torch.randn(shape + (3, 3), generator=g, dtype=torch.float64),
                      torch.randn(shape + (3, 3), generator=g, dtype=torch.float64))
    X = 0.5 * (A - A.transpose(-1, -2).conj())
    tr = torch.diagonal(X, dim1=-2, dim2=-1).sum(-1) / 3
    return X - tr[..., None, None] * torch.eye(3, dtype=X.dtype)


def test_force_full_size_bench_configuration():
    """The 16^3 x 32 differentiation workload at full size with the bench's
    hierarchy: S_f(phi = D xi) = |xi|^2 exactly; the library's force against
    the oracle's force formula on X = (D D^dag)^-1 phi (from the library's
    shifted solve, its residual checked with the oracle's operator) and
    Y = D^dag X (oracle), to the 1e-8 force target; and the force's
    directional derivative -2 sum tr(F w) against central finite differences
    (step 1e-5) of the library's S_f along 16 random su(3) directions.  FD
    bar: S_f is computed to about 1e-14 relative (solves to 1e-12), i.e.
    2e-8 absolute at |xi|^2 = 1.6e6, which the step turns into 1e-3 in the
    difference quotient; the bar is 1e-6 relative plus 1e-2 absolute."""
    import bench
    from oracle import force as oforce
    w = workload("c4")
    m0 = load_m0()[w.name]
    say("c4 full size: inputs", w.dims)
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"]))
    Ud = to_dev(U)
    xi = gaussian_spinor(w.dims, w.seeds["xi"], n=1)
    xid = to_dev(xi)
    p = bench.solver_params(tm, w, tm.MIXED)
    s = tm.Solver(w.dims, p)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    phid = torch.empty_like(xid)
    s.apply(tm.OP_D64, 0, xid, phid, [w.mu])
    F = torch.empty_like(Ud)
    S, info = s.force(phid, F, tol=1e-12)
    xi2 = float((torch.as_tensor(xi).abs() ** 2).sum())
    say(f"  S {S:.15e} |xi|^2 {xi2:.15e} ({info.outer_iters} outer iterations)")
    assert info.status == 0 and abs(S - xi2) / xi2 < 1e-10

    op = WilsonClover(U, m0, w.csw)
    xs = torch.empty_like(phid)
    s.solve_shifted(phid, xs, [0.0], tol=1e-12)
    X = field(xs.cpu()[0])
    phi = field(phid.cpu()[0])
    Y = op.apply_dag(X, w.mu)
    res = norm(phi - op.apply(Y, w.mu)) / norm(phi)
    F_ref = oforce.force_from_fields(U, m0, w.csw, X, Y)
    err = rel(F.cpu(), F_ref)
    say(f"  X residual (oracle operator) {res:.2e}; force vs oracle formula {err:.2e}")
    assert res <= 1e-10 and err < 1e-8

    s_fd = tm.Solver(w.dims, p)
    s_fd.setup(Ud, kappa_of(m0), w.csw, w.mu)
    Fc = F.cpu()
    h = 1e-5
    worst = 0.0
    for k in range(16):
        om = random_su3_directions(tuple(U.shape[:-2]), 2000 + k)
        d_f = oforce.directional_derivative(Fc, om)
        Sx = []
        for t in (h, -h):
            s_fd.setup_update(to_dev(torch.matmul(torch.matrix_exp(t * om), U)), 1)
            Ft = torch.empty_like(Ud)
            St, it = s_fd.force(phid, Ft, tol=1e-12)
            assert it.status == 0
            Sx.append(St)
        d_fd = (Sx[0] - Sx[1]) / (2 * h)
        worst = max(worst, abs(d_f - d_fd) / abs(d_fd))
        say(f"  direction {k}: force {d_f:.9e} finite difference {d_fd:.9e}")
        assert abs(d_f - d_fd) <= 1e-6 * abs(d_fd) + 1e-2
    say(f"  worst relative difference {worst:.2e}")


def _window(a, c, dims, r=2, lead=0):
    """Periodic window of half-width r around site c = (x, y, z, t) of an
    array [lead dims..., T, Z, Y, X, ...]."""
    idx = [((c[m] + torch.arange(-r, r + 1)) % dims[m]).tolist() for m in range(4)]
    sl = (slice(None),) * lead
    out = a[sl + (idx[3],)]
    out = out[sl + (slice(None), idx[2])]
    out = out[sl + (slice(None), slice(None), idx[1])]
    return out[sl + (slice(None), slice(None), slice(None), idx[0])]


def test_stencil_paper_volume_sampled_sites():
    """The fine stencil at the paper's volume 64^3 x 128 (33.5M sites, the
    largest single-GPU workload), FP64 and FP32, in the bench's launch
    configuration, checked at sampled sites (interior and on both time
    boundaries) against the oracle's operator on a 5^4 window around each
    site: its clover term and hops only reach one site away, and the
    time-boundary sign is folded into the window's links.  The links are the
    16^3 x 32 workload's field tiled 4 times in every direction (drawing
    the 64^3 x 128 field takes about 9 minutes on the host); the spinor is
    drawn at full size."""
    w5 = workload("c5")
    w4 = workload("c4")
    dims = w5.dims
    m0 = load_m0()[w5.name]
    say("paper volume stencil: inputs", dims)
    U4 = gauge_links(w4.dims, w4.eps, w4.seeds["links"])
    U = torch.as_tensor(U4).repeat(1, 4, 4, 4, 4, 1, 1)
    psi = torch.as_tensor(gaussian_spinor(dims, w5.seeds["source"], n=1))
    say("  inputs ready", tuple(U.shape), tuple(psi.shape))
    p = tm.default_params(nlevels=1, restart=1, precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    Ud = U.to(DEV)
    s.setup(Ud, kappa_of(m0), w5.csw, w5.mu)
    del Ud
    torch.cuda.empty_cache()
    psid = psi.to(DEV)
    out = torch.empty_like(psid)
    sites = [(0, 0, 0, 0), (63, 63, 63, 127), (17, 5, 40, 64), (3, 62, 1, 1), (31, 32, 33, 126), (50, 9, 22, 0),
             (12, 44, 63, 127), (62, 1, 30, 77)]
    T, Z, Y, X = dims[3], dims[2], dims[1], dims[0]
    for opc, bar, name in ((tm.OP_D64, 1e-13, "FP64"), (tm.OP_D32, 2e-6, "FP32")):
        s.apply(opc, 0, psid, out, [w5.mu])
        torch.cuda.synchronize()
        worst = 0.0
        for c in sites:
            Uw = _window(U, c, dims, lead=1).clone()
            # the link from t = T-1 to t = 0 carries the antiperiodic sign
            for k in range(5):
                if (c[3] - 2 + k) % T == T - 1:
                    Uw[3, k] = -Uw[3, k]
            opw = WilsonClover(Uw, m0, w5.csw, antiperiodic=False)
            ref = opw.apply(field(_window(psi[0], c, dims)), w5.mu)[2, 2, 2, 2]
            got = field(out[0, c[3], c[2], c[1], c[0]].cpu())
            worst = max(worst, float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref)))
        say(f"  {name}: worst relative difference over {len(sites)} sites {worst:.2e}")
        assert worst < bar
    ms = s.time_kernel(tm.K_DSLASH32, 1, 5)
    V = X * Y * Z * T
    say(f"  FP32 stencil {ms:.3f} ms per apply = {768 * V / (ms * 1e-3) / 1e9:.0f} GB/s algorithmic")
    s.close()


@pytest.mark.timeout(1500)
def test_batched_solves_full_size_bench_configuration():
    """The 32^3 x 64 batched workload at full size in the bench's
    configuration (hierarchy, restart 12, HIP-graph replays): 12 point
    sources in one batch and 8 shifted systems (D D^dag + sigma_k) x = b on
    one Gaussian source in another.  Every one of the 20 results is checked
    by the residual that defines it, computed on the host with the oracle's
    FP64 operator on the whole lattice: ||b - D x|| / ||b|| <= 1e-10 for the
    sources, ||b - (D D^dag + sigma) x|| / ||b|| <= 1e-10 for the shifts
    (the library corrects the product residual of its two solves)."""
    import bench
    from lattice_inputs import point_sources, rational_shifts
    w = workload("c3")
    m0 = load_m0()[w.name]
    say("c3 full size: inputs", w.dims)
    U = gauge_links(w.dims, w.eps, w.seeds["links"])
    Ud = to_dev(U)
    npt, nsh = w.extra["n_point"], w.extra["n_shift"]
    bp_h = point_sources(w.dims, w.seeds["source"], npt)
    bp = to_dev(bp_h)
    g1 = gaussian_spinor(w.dims, w.seeds["source"] + 100, n=1)
    bs = to_dev(g1).expand(nsh, *g1.shape[1:]).contiguous()
    sig = [float(x) for x in rational_shifts(nsh)]
    p = bench.solver_params(tm, w, tm.MIXED, 1)
    p.restart = 12
    s = tm.Solver(w.dims, p)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    say("  setup done")
    xp = torch.empty_like(bp)
    ip = s.solve(bp, xp, tol=w.tol)
    xs = torch.empty_like(bs)
    ish = s.solve_shifted(bs, xs, sig, tol=w.tol)
    say(f"  sources: {ip.outer_iters} outer (library residual {ip.true_rel_resid:.2e}), "
        f"shifts: {ish.outer_iters} outer (library product residual {ish.true_rel_resid:.2e})")
    assert ip.status == 0 and ish.status == 0
    assert ish.true_rel_resid <= w.tol
    xp_h, xs_h = xp.cpu(), xs.cpu()
    s.close()
    del Ud, bp, bs, xp, xs
    torch.cuda.empty_cache()

    say("  oracle operator on the whole lattice (clover build)")
    op = WilsonClover(torch.as_tensor(U), m0, w.csw)
    del U
    worst_p = 0.0
    for k in range(npt):
        b = field(torch.as_tensor(bp_h[k]))
        r = float(norm(b - op.apply(field(xp_h[k]), w.mu)) / norm(b))
        worst_p = max(worst_p, r)
        say(f"  source {k}: oracle residual {r:.2e}")
    b = field(torch.as_tensor(g1[0]))
    worst_s = 0.0
    for k in range(nsh):
        x = field(xs_h[k])
        mup = (w.mu ** 2 + sig[k]) ** 0.5
        lhs = op.apply(op.apply_dag(x, mup), mup)
        r = float(norm(b - lhs) / norm(b))
        worst_s = max(worst_s, r)
        say(f"  shift {sig[k]:.1e}: oracle residual of (D D^dag + sigma) x = b {r:.2e}")
    say(f"  worst oracle residual: sources {worst_p:.2e}, shifted systems {worst_s:.2e}")
    assert worst_p <= 1e-10
    assert worst_s <= 1e-10
