"""GPU parity of the fermion force dS_f/dU (S_f = phi^dag (D D^dag)^-1 phi)
against the oracle, through the C ABI.

* force_from_fields: the adjoint kernels alone, on fixed random X and Y, at
  two lattices (the 8^4 two-level workload and a rectangular one) to
  1e-12: every hopping direction, the t-boundary sign and the clover
  insertion are exercised;
* tmamg_force: two multigrid solves plus the kernels, against the oracle
  with dense direct solves on a 4^4 lattice, to the 1e-8 force target.
"""
import pytest
import torch

from lattice_inputs import gauge_links, workload, load_m0
from oracle.dirac import WilsonClover, norm
from oracle import force as oforce
from tests.gpu_common import DEV, links, spinors, kappa_of, rel, field, to_dev

pytestmark = pytest.mark.gpu

tm = pytest.importorskip("paper_1710_06198_amd")


def say(*a):
    print(*a, flush=True)


def solver(dims, precision=None, nlevels=2):
    p = tm.default_params(nlevels=nlevels, precision=tm.FP64 if precision is None else precision)
    return tm.Solver(dims, p)


@pytest.mark.parametrize("dims,eps,csw,seed", [((8, 8, 8, 8), 0.3, 1.0, 1001), ((4, 8, 4, 8), 0.4, 1.57, 1301)])
def test_force_from_fields(dims, eps, csw, seed):
    say("force_from_fields", dims)
    m0 = -0.2
    U, Ud = links(dims, eps, seed)
    s = solver(dims)
    s.setup(Ud, kappa_of(m0), csw, 0.01)
    X, Xd = spinors(dims, seed + 1, 1)
    Y, Yd = spinors(dims, seed + 2, 1)
    F = torch.empty((4,) + tuple(reversed(dims)) + (3, 3), dtype=torch.complex128, device=DEV)
    s.force_from_fields(Xd, Yd, F)
    ref = oforce.force_from_fields(torch.as_tensor(U), m0, csw, field(X[0]), field(Y[0]))
    err = rel(F.cpu(), ref)
    say(f"  rel. difference {err:.2e}")
    assert err < 1e-12


def test_force_end_to_end_dense_oracle():
    dims = (4, 4, 4, 4)
    say("tmamg_force vs dense oracle", dims)
    m0, csw, mu = -0.1, 1.3, 0.02
    U, Ud = links(dims, 0.3, 1401)
    p = tm.default_params(nlevels=2, precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    s.setup(Ud, kappa_of(m0), csw, mu)
    phi, phid = spinors(dims, 1402, 1)
    F = torch.empty((4,) + tuple(reversed(dims)) + (3, 3), dtype=torch.complex128, device=DEV)
    S, info = s.force(phid, F, tol=1e-12)
    say("  info", info.as_dict())
    assert info.status == 0

    Ut = torch.as_tensor(U)
    op = WilsonClover(Ut, m0, csw)
    n = 12 * 4 ** 4
    dense = {sgn: op.dense(sgn * mu) for sgn in (1, -1)}

    def solve(b, mu_tm):
        x = torch.linalg.solve(dense[1 if mu_tm > 0 else -1], b.reshape(n))
        return x.reshape(b.shape)

    S_ref, F_ref, _, _ = oforce.action_and_force(Ut, m0, csw, mu, field(phi[0]), solve)
    say(f"  S {S:.12e} oracle {S_ref:.12e}")
    assert abs(S - S_ref) / abs(S_ref) < 1e-10
    err = rel(F.cpu(), F_ref)
    say(f"  force rel. difference {err:.2e}")
    assert err < 1e-8


def random_su3_directions(shape, seed):
    """Traceless anti-Hermitian 3x3 per link (a direction X of U -> exp(tX) U)."""
    g = torch.Generator().manual_seed(seed)
    A = torch.complex(torch.randn(shape + (3, 3), generator=g, dtype=torch.float64),
                      torch.randn(shape + (3, 3), generator=g, dtype=torch.float64))
    X = 0.5 * (A - A.transpose(-1, -2).conj())
    tr = torch.diagonal(X, dim1=-2, dim2=-1).sum(-1) / 3
    return X - tr[..., None, None] * torch.eye(3, dtype=X.dtype)


def test_autograd_action_gradient():
    """FermionAction (torch.autograd.Function over the library's solves and
    adjoint kernels): U.grad against the oracle's force through dense solves
    (G = 2 F U, to the 1e-8 force target) and against central finite
    differences of the library's own S_f along random su(3) directions
    U -> exp(tX) U (the first-order change is Re sum conj(G) X U)."""
    dims = (4, 4, 4, 4)
    say("autograd action", dims)
    m0, csw, mu = -0.1, 1.3, 0.02
    U, Ud = links(dims, 0.3, 1401)
    p = tm.default_params(nlevels=2, precision=tm.MIXED, storage=tm.STORE_BF16)
    s = tm.Solver(dims, p)
    phi, phid = spinors(dims, 1402, 1)
    Ug = Ud.clone().requires_grad_(True)
    S = tm.fermion_action(Ug, phid, s, kappa_of(m0), csw, mu, tol=1e-12)
    S.backward()
    G = Ug.grad.cpu()

    Ut = torch.as_tensor(U)
    op = WilsonClover(Ut, m0, csw)
    n = 12 * 4 ** 4
    dense = {sgn: op.dense(sgn * mu) for sgn in (1, -1)}

    def solve(b, mu_tm):
        return torch.linalg.solve(dense[1 if mu_tm > 0 else -1], b.reshape(n)).reshape(b.shape)

    S_ref, F_ref, _, _ = oforce.action_and_force(Ut, m0, csw, mu, field(phi[0]), solve)
    G_ref = 2 * torch.matmul(F_ref.contiguous(), Ut.contiguous())
    err = rel(G, G_ref)
    say(f"  S {float(S.detach()):.12e} oracle {S_ref:.12e}; gradient rel. difference {err:.2e}")
    assert abs(float(S.detach()) - S_ref) / abs(S_ref) < 1e-10
    assert err < 1e-8

    s_fd = tm.Solver(dims, p)
    h = 1e-4
    for k in range(2):
        X = random_su3_directions(tuple(Ut.shape[:-2]), 1410 + k)
        d_ad = float((G.conj() * torch.matmul(X, Ut)).real.sum())
        Sp = float(tm.fermion_action(to_dev(torch.matmul(torch.matrix_exp(h * X), Ut)), phid, s_fd,
                                     kappa_of(m0), csw, mu, tol=1e-13))
        Sm = float(tm.fermion_action(to_dev(torch.matmul(torch.matrix_exp(-h * X), Ut)), phid, s_fd,
                                     kappa_of(m0), csw, mu, tol=1e-13))
        d_fd = (Sp - Sm) / (2 * h)
        say(f"  direction {k}: autograd {d_ad:.10e} finite difference {d_fd:.10e}")
        assert abs(d_ad - d_fd) <= 1e-6 * abs(d_fd)
