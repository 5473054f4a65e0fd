"""Pins of the oracle operator D(mu) = D + i mu Gamma5 against what the
mathematics fixes: the free-field momentum-space symbol and spectrum in
closed form, the FFT solve, Gamma5-hermiticity, the twisted-mass bound
D D^dag >= mu^2 (Sec. 1), gauge covariance, the clover term's structure and
an abelian closed form of its leaves, and dense direct solves on 4^4."""
import numpy as np
import pytest
import torch

from lattice_inputs import (gauge_links, gaussian_spinor, unit_links, random_gauge_transform,
                            workload, su3_from_coeffs)
from oracle.dirac import (WilsonClover, gammas, sigma_munu, spinor_to_field, free_field_solve,
                          vdot, norm, clover_term, CDT)

D44 = (4, 4, 4, 4)


def _same_multiset(a, b, tol):
    """Greedy nearest matching of two equally long sets of complex numbers."""
    if len(a) != len(b):
        return False
    key = lambda v: (np.round(v.real / tol / 100), np.round(v.imag / tol / 100))
    rem = list(b)
    for v in sorted(a, key=key):
        j = int(np.argmin(np.abs(np.array(rem) - v)))
        if abs(rem[j] - v) > tol:
            return False
        rem.pop(j)
    return True


def rnd_field(dims, seed, n=None):
    f = spinor_to_field(gaussian_spinor(dims, seed, n=1 if n is None else n))
    return f[0] if n is None else f


# ----------------------------------------------------------------- gammas
def test_gamma_algebra():
    g = gammas().numpy()
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T)
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2 * np.eye(4) * (m == n))
        assert np.allclose(g[4] @ g[m] + g[m] @ g[4], 0)
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))
    sig = sigma_munu().numpy()
    # sigma commutes with g5: the clover term is block diagonal in chirality
    for m in range(4):
        for n in range(4):
            assert np.allclose(sig[m, n] @ g[4], g[4] @ sig[m, n])


def test_links_are_su3():
    U = gauge_links((4, 4, 4, 8), 0.3, 7)
    uu = np.einsum("...ij,...kj->...ik", U, U.conj())
    assert np.abs(uu - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_md_step_links_stay_su3_and_move_by_the_step():
    """The random-walk stand-in for MD updates keeps the links in SU(3) and
    moves each by about step * |g| (the generator norm), so halving the
    step halves the mean distance."""
    from lattice_inputs import md_step_links
    U = gauge_links((4, 4, 4, 4), 0.3, 8)
    for step in (0.05, 0.025):
        V = md_step_links(U, step, 9)
        vv = np.einsum("...ij,...kj->...ik", V, V.conj())
        assert np.abs(vv - np.eye(3)).max() < 1e-14
        assert np.abs(np.linalg.det(V) - 1).max() < 1e-14
    d1 = np.linalg.norm(md_step_links(U, 0.05, 9) - U, axis=(-2, -1)).mean()
    d2 = np.linalg.norm(md_step_links(U, 0.025, 9) - U, axis=(-2, -1)).mean()
    assert abs(d1 / d2 - 2) < 0.01
    assert 0.01 < d1 < 0.2


# ----------------------------------------------------------------- free field
def _symbol_np(p, m0, mu):
    """Momentum-space D at U = 1, derived independently: a plane wave
    e^{ipx} u picks up (1 -/+ g) e^{+-ip}/2 from the two hops."""
    g = gammas().numpy()
    out = (m0 + 4) * np.eye(4, dtype=complex) + 1j * mu * g[4]
    for m in range(4):
        out -= 0.5 * ((np.eye(4) - g[m]) * np.exp(1j * p[m]) + (np.eye(4) + g[m]) * np.exp(-1j * p[m]))
    return out


@pytest.mark.parametrize("n", [(1, 0, 2, 0), (3, 2, 1, 3), (0, 0, 0, 1)])
def test_free_field_plane_wave(n):
    dims = (4, 4, 4, 6)
    m0, mu = -0.3, 0.07
    op = WilsonClover(unit_links(dims), m0, 1.3)
    p = [2 * np.pi * n[0] / dims[0], 2 * np.pi * n[1] / dims[1], 2 * np.pi * n[2] / dims[2],
         2 * np.pi * (n[3] + 0.5) / dims[3]]
    t, z, y, x = np.meshgrid(*[np.arange(dims[3 - i]) for i in range(4)], indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = torch.tensor((phase[..., None, None] * u).reshape(*phase.shape, 12))
    out = op.apply(psi, mu)
    expect = phase[..., None, None] * (_symbol_np(p, m0, mu) @ u)
    assert np.abs(out.numpy() - expect.reshape(out.shape)).max() < 1e-13
    # closed-form eigenvalues a(p) +- i sqrt(sum sin^2 + mu^2)
    a = m0 + sum(1 - np.cos(pm) for pm in p)
    r = np.sqrt(sum(np.sin(pm) ** 2 for pm in p) + mu * mu)
    ev = np.linalg.eigvals(_symbol_np(p, m0, mu))
    assert _same_multiset(ev, np.array([a - 1j * r, a - 1j * r, a + 1j * r, a + 1j * r]), 1e-12)


def test_free_field_dense_spectrum():
    dims = D44
    m0, mu = 0.1, 0.05
    op = WilsonClover(unit_links(dims), m0, 1.0)
    ev = np.linalg.eigvals(op.dense(mu).numpy())
    exp = []
    for nt in range(4):
        for nz in range(4):
            for ny in range(4):
                for nx in range(4):
                    p = [2 * np.pi * nx / 4, 2 * np.pi * ny / 4, 2 * np.pi * nz / 4, 2 * np.pi * (nt + .5) / 4]
                    a = m0 + sum(1 - np.cos(q) for q in p)
                    r = np.sqrt(sum(np.sin(q) ** 2 for q in p) + mu * mu)
                    exp += [a + 1j * r] * 6 + [a - 1j * r] * 6
    assert _same_multiset(ev, np.array(exp), 1e-10)


@pytest.mark.parametrize("name", ["c1", "c4", "c2"])
def test_free_field_fft_solve_full_volume(name):
    w = workload(name)
    m0 = -0.2
    op = WilsonClover(unit_links(w.dims), m0, w.csw)
    b = rnd_field(w.dims, 11)
    x = free_field_solve(b, m0, w.mu)
    assert norm(op.apply(x, w.mu) - b) / norm(b) < 1e-12


def test_free_field_smallest_real_part():
    # free operator at m0 = 0, mu = 0: smallest real part is 1 - cos(pi/Lt)
    from oracle.mcrit import smallest_real_part
    dims = (4, 4, 4, 6)
    lam = smallest_real_part(unit_links(dims), 1.0, ncv=40, tol=1e-10)
    assert abs(lam.real - (1 - np.cos(np.pi / 6))) < 1e-8


# ----------------------------------------------------------------- identities
@pytest.fixture(scope="module")
def rough_op():
    U = gauge_links(D44, 0.4, 21)
    return WilsonClover(U, -0.35, 1.7)


def test_gamma5_hermiticity(rough_op):
    psi, chi = rnd_field(D44, 1), rnd_field(D44, 2)
    mu = 0.031
    lhs = vdot(psi, rough_op.g5 * rough_op.apply(rough_op.g5 * chi, mu))
    rhs = vdot(rough_op.apply(psi, -mu), chi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_norm_identity_and_bound(rough_op):
    """||D(mu) psi||^2 = ||D(0) psi||^2 + mu^2 ||psi||^2, hence D D^dag >= mu^2."""
    psi = rnd_field(D44, 3)
    for mu in (0.0, 0.01, 0.3):
        a = norm(rough_op.apply(psi, mu)) ** 2
        b = norm(rough_op.apply(psi, 0.0)) ** 2 + mu * mu * norm(psi) ** 2
        assert abs(a - b) < 1e-13 * a


def test_dense_smallest_singular_value(rough_op):
    mu = 0.02
    s = torch.linalg.svdvals(rough_op.dense(mu))
    assert s.min().item() >= mu * (1 - 1e-12)


def test_dense_lu_solve(rough_op):
    mu = 0.02
    b = rnd_field(D44, 4)
    M = rough_op.dense(mu)
    x = torch.linalg.solve(M, b.reshape(-1)).reshape(b.shape)
    assert norm(rough_op.apply(x, mu) - b) / norm(b) < 1e-13
    # the dense matrix is D itself: its action equals the stencil's
    assert norm((M @ b.reshape(-1)).reshape(b.shape) - rough_op.apply(b, mu)) < 1e-12 * norm(b)


def test_free_dense_solve_matches_fft():
    op = WilsonClover(unit_links(D44), 0.05, 1.0)
    b = rnd_field(D44, 5)
    x = torch.linalg.solve(op.dense(0.01), b.reshape(-1)).reshape(b.shape)
    y = free_field_solve(b, 0.05, 0.01)
    assert norm(x - y) / norm(y) < 1e-12


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    U = torch.tensor(gauge_links(dims, 0.5, 31))
    G = torch.tensor(random_gauge_transform(dims, 32))
    from oracle.dirac import lshift, dag
    UG = torch.stack([G @ U[m] @ dag(lshift(G, m, 1)) for m in range(4)])
    op, opg = WilsonClover(U, -0.2, 1.5), WilsonClover(UG, -0.2, 1.5)
    psi = rnd_field(dims, 6)

    def gmul(f):
        return torch.einsum("...ab,...sb->...sa", G, f.reshape(*f.shape[:-1], 4, 3)).reshape(f.shape)

    assert norm(opg.apply(gmul(psi), 0.1) - gmul(op.apply(psi, 0.1))) < 1e-12 * norm(psi) * 10
    # A[U^G](x) = G A G^dag in colour
    Gk = torch.einsum("ab,...cd->...acbd", torch.eye(4, dtype=CDT), G).reshape(*G.shape[:-2], 12, 12)
    assert (opg.A - Gk @ op.A @ Gk.conj().transpose(-1, -2)).abs().max() < 1e-12


# ----------------------------------------------------------------- clover
def test_clover_structure(rough_op):
    A = rough_op.A - (rough_op.m0 + 4) * torch.eye(12, dtype=CDT)
    assert (A - A.conj().transpose(-1, -2)).abs().max() < 1e-14
    assert A[..., :6, 6:].abs().max() < 1e-15 and A[..., 6:, :6].abs().max() < 1e-15
    assert A.abs().max() > 1e-2
    op1 = WilsonClover(unit_links(D44), 0.3, 2.0)
    assert (op1.A - 4.3 * torch.eye(12, dtype=CDT)).abs().max() == 0


def test_clover_abelian_closed_form():
    """U_mu(x) = exp(i theta_mu(x) T), T = diag(1,-1,0): every leaf is
    exp(i Theta T) with Theta its lattice curl, so Fhat_{mu nu} equals
    (i/4) sum_leaves sin(Theta_leaf) T exactly."""
    dims = (4, 6, 4, 4)
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(9)
    th = rng.uniform(-1.0, 1.0, size=(4, lt, lz, ly, lx))
    Tm = np.diag([1.0, -1.0, 0.0])
    U = np.zeros((4, lt, lz, ly, lx, 3, 3), complex)
    for k, v in enumerate([1.0, -1.0, 0.0]):
        U[..., k, k] = np.exp(1j * th * v)
    ax = {0: 3, 1: 2, 2: 1, 3: 0}

    def sh(a, m, s):  # a(x + s*m)
        return np.roll(a, -s, axis=ax[m])

    csw = 1.3
    expect = np.zeros((lt, lz, ly, lx, 12, 12), complex)
    sig = sigma_munu().numpy()
    for m in range(4):
        for n in range(4):
            if m == n:
                continue
            tm, tn = th[m], th[n]
            leaves = [
                tm + sh(tn, m, 1) - sh(tm, n, 1) - tn,
                tn - sh(sh(tm, m, -1), n, 1) - sh(tn, m, -1) + sh(tm, m, -1),
                -sh(tm, m, -1) - sh(sh(tn, m, -1), n, -1) + sh(sh(tm, m, -1), n, -1) + sh(tn, n, -1),
                -sh(tn, n, -1) + sh(tm, n, -1) + sh(sh(tn, n, -1), m, 1) - tm,
            ]
            fhat = 0.25j * sum(np.sin(L) for L in leaves)
            F = fhat[..., None, None] * Tm
            expect += np.einsum("ab,...cd->...acbd", sig[m, n], F).reshape(lt, lz, ly, lx, 12, 12)
    expect *= csw * 0.25j
    got = clover_term(torch.tensor(U), csw).numpy()
    assert np.abs(got - expect).max() < 1e-14


# ----------------------------------------------------------------- even-odd reduction
def test_schur_complement_reproduces_dense_solve():
    """The even-odd reduction pinned against a dense solve of the full system
    on 4^4: the even part of x = D^-1 b satisfies D_hat x_e = b_e - D_eo
    D_oo^-1 b_o, and x_o = D_oo^-1 (b_o - D_oe x_e) gives back the odd part;
    both for mu = 0 and a twisted mass, with a nontrivial clover term."""
    from oracle.evenodd import SchurOperator
    dims = (4, 4, 4, 4)
    U = torch.tensor(gauge_links(dims, 0.4, 41))
    op = WilsonClover(U, -0.2, 1.7)
    b = spinor_to_field(gaussian_spinor(dims, 42)[0])
    n = 12 * 4 ** 4
    for mu in (0.0, 0.07):
        x = torch.linalg.solve(op.dense(mu), b.reshape(n)).reshape(b.shape)
        S = SchurOperator(op, mu)
        lhs = S.apply(x)
        rhs = S.reduced_rhs(b)
        assert float((lhs - rhs).abs().max()) < 1e-12 * float(rhs.abs().max())
        xo = S.odd_solution(b, x)
        assert float((xo - x * S.odd).abs().max()) < 1e-12 * float(x.abs().max())


def test_schur_operator_ignores_odd_input_and_is_gamma5_compatible():
    """Odd-site input entries do not change D_hat psi, its odd outputs are 0,
    and D_hat(mu)^dag = Gamma5 D_hat(-mu) Gamma5 (inherited from D)."""
    from oracle.evenodd import SchurOperator
    dims = (4, 4, 4, 4)
    U = torch.tensor(gauge_links(dims, 0.4, 43))
    op = WilsonClover(U, -0.1, 1.3)
    a = spinor_to_field(gaussian_spinor(dims, 44)[0])
    c = spinor_to_field(gaussian_spinor(dims, 45)[0])
    Sp, Sm = SchurOperator(op, 0.05), SchurOperator(op, -0.05)
    assert torch.allclose(Sp.apply(a), Sp.apply(a * Sp.even), atol=0, rtol=0)
    assert float((Sp.apply(a) * Sp.odd).abs().max()) == 0.0
    ae, ce = a * Sp.even, c * Sp.even
    lhs = torch.sum(ce.conj() * Sp.apply(ae))
    rhs = torch.sum((op.g5 * Sm.apply(op.g5 * ce)).conj() * ae)
    assert abs(complex(lhs - rhs)) < 1e-11 * abs(complex(lhs))
