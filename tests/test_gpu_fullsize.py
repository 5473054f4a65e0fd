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


def test_batched_solves_full_size_bench_configuration():
    """The 32^3 x 64 batched workload at full size in the bench's
    configuration (hierarchy, restart 12, HIP-graph replays): 12 point
    sources in one batch and 8 shifted systems (D D^dag + sigma_k) x = b on
    one Gaussian source in another.  The results are checked by the
    residuals that define them, computed with the library's FP64 stencil,
    which is itself checked against the oracle at sampled sites of this
    lattice (5^4 windows, as for the paper-volume stencil test):
    ||b - D x|| / ||b|| <= 1e-10 for every source; for the shifts the two
    solves of 1e-10 each bound the residual of the product by about
    ||D|| 1e-10 / mu'_min = 8e-10 / 3.5e-3 = 2.3e-7, bar 5e-7."""
    import bench
    from lattice_inputs import point_sources, rational_shifts
    w = workload("c3")
    m0 = load_m0()[w.name]
    say("c3 full size: inputs", w.dims)
    U = gauge_links(w.dims, w.eps, w.seeds["links"])
    Ud = to_dev(U)
    npt, nsh = w.extra["n_point"], w.extra["n_shift"]
    bp = to_dev(point_sources(w.dims, w.seeds["source"], npt))
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
    say(f"  sources: {ip.outer_iters} outer, shifts: {ish.outer_iters} outer")
    assert ip.status == 0 and ish.status == 0

    # the library's FP64 stencil against the oracle at sampled sites, on
    # the Gaussian source (a solution would make D x ~ b = 0 away from a
    # point source: cancellation to the residual level)
    Dx = torch.empty_like(bs[:1])
    s.apply(tm.OP_D64, 0, bs[:1], Dx, [w.mu])
    x0 = torch.as_tensor(g1[0])
    Ut = torch.as_tensor(U)
    T = w.dims[3]
    worst = 0.0
    for c in [(0, 0, 0, 0), (31, 31, 31, 63), (5, 17, 29, 40), (12, 3, 8, 0)]:
        Uw = _window(Ut, c, w.dims, lead=1).clone()
        for k in range(5):
            if (c[3] - 2 + k) % T == T - 1:
                Uw[3, k] = -Uw[3, k]
        ref = WilsonClover(Uw, m0, w.csw, antiperiodic=False).apply(field(_window(x0, c, w.dims)), w.mu)[2, 2, 2, 2]
        got = field(Dx[0, c[3], c[2], c[1], c[0]].cpu())
        worst = max(worst, float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref)))
    say(f"  FP64 stencil at sampled sites vs oracle: {worst:.2e}")
    assert worst < 1e-13

    # residuals with the library's FP64 stencil
    def rel_res(b, r):
        return float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))

    Dxp = torch.empty_like(xp)
    s.apply(tm.OP_D64, 0, xp, Dxp, [w.mu] * npt)
    res_p = max(rel_res(bp[k], bp[k] - Dxp[k]) for k in range(npt))
    g5 = torch.tensor([1, 1, -1, -1], dtype=torch.complex128, device=xs.device).reshape(4, 1)
    mup = [(w.mu ** 2 + sg) ** 0.5 for sg in sig]
    z = torch.empty_like(xs)
    s.apply(tm.OP_D64, 0, (g5 * xs).contiguous(), z, [-m for m in mup])
    y = torch.empty_like(xs)
    s.apply(tm.OP_D64, 0, (g5 * z).contiguous(), y, mup)
    res_s = max(rel_res(bs[k], bs[k] - y[k]) for k in range(nsh))
    say(f"  worst residual: sources {res_p:.2e}, shifted systems {res_s:.2e}")
    assert res_p <= 1e-10
    assert res_s <= 5e-7
    s.close()
