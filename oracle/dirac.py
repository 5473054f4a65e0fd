"""Oracle: the twisted-mass clover Wilson operator D(mu) = D + i mu Gamma5.

The paper (Sec. 1 and Sec. 1.1) works with the clover-improved Wilson
operator D and its twisted-mass form D(+-mu) = D +- i mu Gamma5; it states
that the twisted-mass term bounds D D^dag from below by mu^2.  It does not
print D itself; the standard definition used here (m0-normalised):

  D(mu) psi(x) = A(x) psi(x) + i mu g5 psi(x)
     - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]

  A(x) = (m0 + 4) + c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),
  Fhat = (Q_{mu nu} - Q_{mu nu}^dag)/8 made traceless, Q = sum of the four
  plaquette leaves anchored at x, sigma_{mu nu} = (i/2)[g_mu, g_nu].

Chiral gamma basis: g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]],
g5 = g1 g2 g3 g4 = diag(1, 1, -1, -1).  Fields are periodic in space and
antiperiodic in time; the sign is applied to hops across the time boundary
only (never to the plaquettes, where it would cancel).

Fields: torch complex128 [..., T, Z, Y, X, 12] with spin-colour index
s*3 + c.  Links: complex128 [4, T, Z, Y, X, 3, 3], mu = 0..3 <-> x, y, z, t.
"""
from __future__ import annotations

import numpy as np
import torch

CDT = torch.complex128


def gammas() -> torch.Tensor:
    """[5, 4, 4]: g_1..g_4 (x, y, z, t) then g5, chiral basis."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
         np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    e = np.eye(2, dtype=complex)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.block([[z, e], [e, z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    g.append(g5)
    return torch.tensor(np.array(g), dtype=CDT)


def sigma_munu() -> torch.Tensor:
    """[4, 4, 4, 4]: sigma_{mu nu} = (i/2)[g_mu, g_nu]."""
    g = gammas()
    sig = torch.zeros(4, 4, 4, 4, dtype=CDT)
    for m in range(4):
        for n in range(4):
            sig[m, n] = 0.5j * (g[m] @ g[n] - g[n] @ g[m])
    return sig


def gamma5_dof(d: int) -> torch.Tensor:
    """Gamma5 on a level with d dof per site: +1 on the first half, -1 on the second.

    On the fine level (d = 12, index s*3 + c) this is g5 = diag(1,1,-1,-1) x I_3;
    on a coarse level it is Gamma5,c = diag(I_Nv, -I_Nv) (Sec. 1.1).
    """
    g = torch.ones(d, dtype=torch.float64)
    g[d // 2:] = -1
    return g


# ---------------------------------------------------------------- shifts
def _axis(mu: int, xaxis: int) -> int:
    return xaxis - mu


def shift(f: torch.Tensor, mu: int, step: int, xaxis: int, antiperiodic: bool = False):
    """f(x + step*mu_hat) on a periodic lattice; optional -1 on t-wraps.

    xaxis is the (negative) tensor axis of the x coordinate; y, z, t follow
    to its left.
    """
    ax = _axis(mu, xaxis)
    out = torch.roll(f, shifts=-step, dims=ax)
    if antiperiodic and mu == 3:
        lt = f.shape[ax]
        sign = torch.ones(lt, dtype=torch.float64)
        if step > 0:
            sign[lt - 1] = -1.0      # x + t_hat wraps from t = Lt-1 to t = 0
        else:
            sign[0] = -1.0           # x - t_hat wraps from t = 0 to t = Lt-1
        shape = [1] * f.dim()
        shape[ax] = lt
        out = out * sign.reshape(shape)
    return out


def lshift(u: torch.Tensor, mu: int, step: int) -> torch.Tensor:
    """A link/colour-matrix field [..., T, Z, Y, X, 3, 3] at x + step*mu_hat."""
    return shift(u, mu, step, xaxis=-3)


def dag(m: torch.Tensor) -> torch.Tensor:
    return m.conj().transpose(-1, -2)


# ---------------------------------------------------------------- clover
def clover_leaves(U: torch.Tensor, mu: int, nu: int) -> torch.Tensor:
    """Q_{mu nu}(x): sum of the four plaquettes in the (mu, nu) plane anchored
    at x, all with the same orientation (mu then nu)."""
    Um, Un = U[mu], U[nu]
    l1 = Um @ lshift(Un, mu, 1) @ dag(lshift(Um, nu, 1)) @ dag(Un)
    Um_mm = lshift(Um, mu, -1)
    Un_mm = lshift(Un, mu, -1)
    l2 = Un @ dag(lshift(Um_mm, nu, 1)) @ dag(Un_mm) @ Um_mm
    Um_mm_mn = lshift(Um_mm, nu, -1)
    Un_mm_mn = lshift(Un_mm, nu, -1)
    l3 = dag(Um_mm) @ dag(Un_mm_mn) @ Um_mm_mn @ lshift(Un, nu, -1)
    Un_mn = lshift(Un, nu, -1)
    Um_mn = lshift(Um, nu, -1)
    l4 = dag(Un_mn) @ Um_mn @ lshift(Un_mn, mu, 1) @ dag(Um)
    return l1 + l2 + l3 + l4


def field_strength(U: torch.Tensor, mu: int, nu: int, traceless: bool = True):
    """Fhat_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/8, optionally traceless."""
    q = clover_leaves(U, mu, nu)
    f = (q - dag(q)) / 8.0
    if traceless:
        tr = torch.diagonal(f, dim1=-2, dim2=-1).sum(-1)
        eye = torch.eye(3, dtype=CDT)
        f = f - (tr / 3.0)[..., None, None] * eye
    return f


def clover_term(U: torch.Tensor, csw: float) -> torch.Tensor:
    """c_sw (i/4) sum_{mu,nu} sigma_{mu nu} x Fhat_{mu nu}: [T, Z, Y, X, 12, 12]."""
    sig = sigma_munu()
    dims = U.shape[1:5]
    out = torch.zeros(*dims, 12, 12, dtype=CDT)
    for m in range(4):
        for n in range(4):
            if m == n:
                continue
            f = field_strength(U, m, n)
            # kron(sigma, F) with index s*3 + c
            k = torch.einsum("ab,...cd->...acbd", sig[m, n], f).reshape(*dims, 12, 12)
            out = out + k
    return (csw * 0.25j) * out


# ---------------------------------------------------------------- operator
class WilsonClover:
    """D(mu) on the fine lattice; psi: [..., T, Z, Y, X, 12] complex128."""

    dof = 12

    def __init__(self, U, m0: float, csw: float, antiperiodic: bool = True):
        self.U = torch.as_tensor(U, dtype=CDT)
        self.m0 = float(m0)
        self.csw = float(csw)
        self.antiperiodic = antiperiodic
        lt, lz, ly, lx = self.U.shape[1:5]
        self.dims = (lx, ly, lz, lt)
        self.A = clover_term(self.U, self.csw)
        eye = torch.eye(12, dtype=CDT)
        self.A = self.A + (self.m0 + 4.0) * eye
        g = gammas()
        e4 = torch.eye(4, dtype=CDT)
        self.proj_m = [(e4 - g[m]) for m in range(4)]   # 1 - g_mu (forward hop)
        self.proj_p = [(e4 + g[m]) for m in range(4)]   # 1 + g_mu (backward hop)
        self.g5 = gamma5_dof(12)

    # building blocks; each maps a field to a field
    def diag(self, psi, mu_tm: float = 0.0):
        out = torch.einsum("...ij,...j->...i", self.A, psi)
        if mu_tm != 0.0:
            out = out + 1j * mu_tm * self.g5 * psi
        return out

    def _spin_colour(self, proj, u, psi):
        p = psi.reshape(*psi.shape[:-1], 4, 3)
        up = torch.einsum("...ab,...sb->...sa", u, p)
        out = torch.einsum("st,...tc->...sc", proj, up)
        return out.reshape(psi.shape)

    def hop(self, psi, mu: int, direction: int):
        """Hopping term towards x + direction*mu_hat, including the -1/2."""
        if direction > 0:
            src = shift(psi, mu, +1, xaxis=-2, antiperiodic=self.antiperiodic)
            return -0.5 * self._spin_colour(self.proj_m[mu], self.U[mu], src)
        src = shift(psi, mu, -1, xaxis=-2, antiperiodic=self.antiperiodic)
        ub = dag(lshift(self.U[mu], mu, -1))
        return -0.5 * self._spin_colour(self.proj_p[mu], ub, src)

    def apply(self, psi, mu_tm: float = 0.0):
        out = self.diag(psi, mu_tm)
        for m in range(4):
            out = out + self.hop(psi, m, +1) + self.hop(psi, m, -1)
        return out

    def apply_dag(self, psi, mu_tm: float = 0.0):
        """D(mu)^dag = Gamma5 D(-mu) Gamma5."""
        return self.g5 * self.apply(self.g5 * psi, -mu_tm)

    def dense(self, mu_tm: float = 0.0) -> torch.Tensor:
        """Dense matrix of D(mu) (only for tiny lattices)."""
        lx, ly, lz, lt = self.dims
        n = lx * ly * lz * lt * 12
        eye = torch.eye(n, dtype=CDT).reshape(n, lt, lz, ly, lx, 12)
        cols = self.apply(eye, mu_tm).reshape(n, n)
        return cols.T.contiguous()


# ---------------------------------------------------------------- free field
def free_field_symbol(p, m0: float, mu_tm: float) -> torch.Tensor:
    """Momentum-space D(mu) at U = 1: a(p) + i sum g_mu sin p_mu + i mu g5."""
    g = gammas()
    a = m0 + sum(1.0 - np.cos(pm) for pm in p)
    out = a * torch.eye(4, dtype=CDT) + 1j * mu_tm * g[4]
    for m in range(4):
        out = out + 1j * np.sin(p[m]) * g[m]
    return out


def free_field_solve(b: torch.Tensor, m0: float, mu_tm: float) -> torch.Tensor:
    """x = D(mu)^-1 b at U = 1 in closed form by FFT.

    Antiperiodic time: the phase e^{-i pi t/Lt} makes the field periodic;
    momenta are p_i = 2 pi n_i / L_i, p_t = 2 pi (n_t + 1/2) / L_t.
    D^-1(p) = (a - i sum g sin p - i mu g5) / (a^2 + sum sin^2 p + mu^2).
    b: [T, Z, Y, X, 12].
    """
    lt, lz, ly, lx = b.shape[:4]
    t = torch.arange(lt, dtype=torch.float64)
    ph = torch.exp(-1j * np.pi * t / lt).to(CDT).reshape(lt, 1, 1, 1, 1)
    f = torch.fft.fftn(b * ph, dim=(0, 1, 2, 3))
    g = gammas()
    kt = 2 * np.pi * (torch.arange(lt, dtype=torch.float64) + 0.5) / lt
    kz = 2 * np.pi * torch.arange(lz, dtype=torch.float64) / lz
    ky = 2 * np.pi * torch.arange(ly, dtype=torch.float64) / ly
    kx = 2 * np.pi * torch.arange(lx, dtype=torch.float64) / lx
    PT, PZ, PY, PX = torch.meshgrid(kt, kz, ky, kx, indexing="ij")
    ps = [PX, PY, PZ, PT]
    a = m0 + sum(1.0 - torch.cos(pm) for pm in ps)
    s2 = sum(torch.sin(pm) ** 2 for pm in ps)
    den = a * a + s2 + mu_tm * mu_tm
    inv = a[..., None, None] * torch.eye(4, dtype=CDT) - 1j * mu_tm * g[4]
    for m in range(4):
        inv = inv - 1j * torch.sin(ps[m])[..., None, None] * g[m]
    inv = inv / den[..., None, None]
    ff = f.reshape(lt, lz, ly, lx, 4, 3)
    xf = torch.einsum("...st,...tc->...sc", inv, ff).reshape(lt, lz, ly, lx, 12)
    x = torch.fft.ifftn(xf, dim=(0, 1, 2, 3))
    return x / ph


def spinor_to_field(psi_np) -> torch.Tensor:
    """canonical [..., T, Z, Y, X, 4, 3] -> oracle field [..., T, Z, Y, X, 12]."""
    t = torch.as_tensor(psi_np, dtype=CDT)
    return t.reshape(*t.shape[:-2], 12)


def field_to_spinor(f: torch.Tensor) -> torch.Tensor:
    return f.reshape(*f.shape[:-1], 4, 3)


def vdot(a: torch.Tensor, b: torch.Tensor) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(torch.sum(a.conj() * b))


def norm(a: torch.Tensor) -> float:
    return float(torch.sqrt(torch.sum((a.conj() * a).real)))
