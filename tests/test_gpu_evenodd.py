"""The even-odd reduced solve (tmamg_solve_eo): D_hat(mu) x_e = b_e on the
even sites, D_hat = D_ee - D_eo D_oo^-1 D_oe, checked by its residual in the
oracle's Schur operator (pinned against a dense solve of the full system),
in both precisions, with signed per-RHS mu; and the full solution rebuilt
from x_e through the oracle's odd-site back substitution solves D x = b."""
import pytest
import torch

from lattice_inputs import workload, load_m0
from oracle.dirac import WilsonClover, norm
from oracle.evenodd import SchurOperator, parity_mask
from tests.gpu_common import links, spinors, kappa_of, field, to_dev

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_even_odd_reduced_solve(precision):
    w = workload("c1")
    m0 = load_m0()["c1"]
    U, Ud = links(w.dims, w.eps, w.seeds["links"])
    op = WilsonClover(U, m0, w.csw)
    p = tm.default_params(nlevels=2, agg=w.agg, nv=w.nv, setup_iters=w.setup_iters, init_smooth=w.init_smooth,
                          sap_sweeps=w.sap_sweeps, mr_steps=w.mr_steps, restart=w.restart,
                          precision=tm.MIXED if precision == "mixed" else tm.FP64, storage=tm.STORE_BF16)
    s = tm.Solver(w.dims, p)
    s.setup(Ud, kappa_of(m0), w.csw, w.mu)
    b, bd = spinors(w.dims, 7901, 2)
    mus = [w.mu, -0.02]
    x = torch.empty_like(bd)
    info = s.solve_eo(bd, x, mus, tol=1e-10)
    say(f"even-odd solve c1 {precision}: {info.outer_iters} outer iterations, library residual "
        f"{info.true_rel_resid:.2e}")
    assert info.status == 0
    even = parity_mask(w.dims, 0)[..., None]
    for r in range(2):
        S = SchurOperator(op, mus[r])
        be = field(b[r]) * even
        xe = field(x.cpu()[r])
        assert float(norm(xe * (1 - even))) == 0.0          # odd sites of x are zero
        res = float(norm(be - S.apply(xe)) / norm(be))
        say(f"  rhs {r} mu {mus[r]}: oracle reduced residual {res:.2e}")
        assert res <= 1e-10
        # with x_o from the odd back substitution, (x_e, x_o) solves D x = (b_e, 0)
        xo = S.odd_solution(be, xe)
        full = float(norm(op.apply(xe + xo, mus[r]) - be) / norm(be))
        assert full <= 1e-9
    s.close()
