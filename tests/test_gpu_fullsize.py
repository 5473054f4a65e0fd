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
