"""The combined workload at the paper's volume, 64^3 x 128 (33.5M sites,
the largest single-GPU case): setup, four Gaussian right-hand sides and the
force, all in one GPU's memory with the bench's memory plan.

Checks: every solve's FP64 true residual (the library's own FP64 operator,
whole lattice) <= 1e-10; the oracle's operator on t-slabs around both time
boundaries and in the middle of the lattice reproduces that residual (the
slab is cut from the full field with one halo slice on each side and the
antiperiodic sign folded into the link that crosses the boundary; the
window method reproduces the full-lattice oracle exactly on a small
lattice, see test_gpu_fullsize); S_f(phi = D xi) = |xi|^2; and the force at
sampled links against the oracle's force formula on a 7^4 window (the
force on U_mu(x) involves X and Y up to two sites from x per direction and
Y there the links one site further), with X = (D D^dag)^-1 phi from the
library's shifted solve and Y = D^dag X from the oracle on the window."""
import os

import pytest
import torch

from lattice_inputs import workload, load_m0, gauge_links, gaussian_spinor
from oracle.dirac import WilsonClover, norm
from tests.gpu_common import DEV, kappa_of, field

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


def _slab(a, t0, t1, T, lead=0):
    """Slices t0 .. t1 - 1 (wrapping) of an array [lead..., T, ...]."""
    idx = [t % T for t in range(t0, t1)]
    return a[(slice(None),) * lead + (idx,)]


def _window(a, c, dims, r, lead=0):
    """Periodic window of half-width r around site c = (x, y, z, t)."""
    idx = [((c[m] + torch.arange(-r, r + 1)) % dims[m]).tolist() for m in range(4)]
    sl = (slice(None),) * lead
    out = a[sl + (idx[3],)]
    out = out[sl + (slice(None), idx[2])]
    out = out[sl + (slice(None), slice(None), idx[1])]
    return out[sl + (slice(None), slice(None), slice(None), idx[0])]


def _fold_time_sign(Uw, t_first, T):
    """The link from t = T - 1 to t = 0 carries the antiperiodic sign."""
    for k in range(Uw.shape[1]):
        if (t_first + k) % T == T - 1:
            Uw[3, k] = -Uw[3, k]
    return Uw


@pytest.mark.timeout(1800)
def test_paper_volume_combined_workload():
    import gc
    import bench
    from oracle import force as oforce
    # the job needs 260 GB of the GPU: return what earlier tests left cached
    gc.collect()
    torch.cuda.empty_cache()
    w = workload("c5")
    m0 = load_m0()[w.name]
    dims = w.dims
    X_, Y_, Z_, T = dims
    nrhs = w.extra.get("nrhs", 4)
    workers = max(1, min(16, os.cpu_count() or 1))
    say("paper volume", dims, f": drawing links ({workers} processes)")
    U = torch.as_tensor(gauge_links(dims, w.eps, w.seeds["links"], workers=workers))
    say("  links drawn")
    s = tm.Solver(dims, bench.paper_volume_params(tm, w))
    Ud = U.to(DEV)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    del Ud
    torch.cuda.empty_cache()
    say(f"  setup done; peak device memory {torch.cuda.max_memory_allocated() / 1e9:.1f} GB")

    b_all = torch.as_tensor(gaussian_spinor(dims, w.seeds["source"], n=nrhs))
    x_all = torch.empty_like(b_all)
    for r in range(nrhs):
        b = b_all[r:r + 1].to(DEV)
        x = torch.empty_like(b)
        info = s.solve(b, x, tol=w.tol)
        say(f"  rhs {r}: {info.outer_iters} outer iterations, library FP64 residual {info.true_rel_resid:.2e}")
        assert info.status == 0 and info.true_rel_resid <= 1e-10
        x_all[r] = x[0].cpu()
        del b, x
    torch.cuda.empty_cache()

    # oracle residual on t-slabs: 4 slices each (both time boundaries and the middle)
    for t0 in (T - 2, T // 2 - 2):
        Uw = _fold_time_sign(_slab(U, t0 - 1, t0 + 5, T, lead=1).clone(), t0 - 1, T)
        opw = WilsonClover(Uw, m0, w.csw, antiperiodic=False)
        for r in range(nrhs):
            bn = norm(field(b_all[r]))
            xw = field(_slab(x_all[r], t0 - 1, t0 + 5, T))
            rw = field(_slab(b_all[r], t0, t0 + 4, T)) - opw.apply(xw, w.mu)[1:5]
            rel = norm(rw) / bn
            say(f"  slab t = {t0 % T} .. {(t0 + 3) % T}, rhs {r}: oracle residual on the slab / |b| {rel:.2e}")
            assert rel <= 1e-10
        del opw, Uw

    # force: S_f(phi = D xi) = |xi|^2, F against the oracle formula at sampled links
    xi = torch.as_tensor(gaussian_spinor(dims, w.seeds["xi"], n=1))
    xid = xi.to(DEV)
    phid = torch.empty_like(xid)
    s.apply(tm.OP_D64, 0, xid, phid, [w.mu])
    del xid
    F = torch.empty((4, T, Z_, Y_, X_, 3, 3), dtype=torch.complex128, device=DEV)
    S, finfo = s.force(phid, F, tol=w.tol)
    xi2 = float((xi.abs() ** 2).sum())
    say(f"  force: S {S:.12e} |xi|^2 {xi2:.12e}, {finfo.outer_iters} outer iterations")
    assert finfo.status == 0 and abs(S - xi2) / xi2 < 1e-9
    Fc = F.cpu()
    del F
    torch.cuda.empty_cache()
    xs = torch.empty_like(phid)
    sinfo = s.solve_shifted(phid, xs, [0.0], tol=w.tol)
    assert sinfo.status == 0
    Xf = xs.cpu()[0]
    del xs, phid
    sites = [(0, 0, 0, 0), (63, 63, 63, 127), (17, 5, 40, 64), (31, 32, 33, 126)]
    worst = 0.0
    for c in sites:
        Uw = _fold_time_sign(_window(U, c, dims, 3, lead=1).clone(), c[3] - 3, T)
        opw = WilsonClover(Uw, m0, w.csw, antiperiodic=False)
        Xw = field(_window(Xf, c, dims, 3))
        Yw = opw.apply_dag(Xw, w.mu)
        Fw = oforce.force_from_fields(Uw, m0, w.csw, Xw, Yw, antiperiodic=False)
        ref = Fw[:, 3, 3, 3, 3]
        got = Fc[:, c[3], c[2], c[1], c[0]]
        err = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))
        worst = max(worst, err)
        say(f"  force at {c}: rel. difference from the oracle formula {err:.2e}")
    assert worst < 1e-8
    s.close()
