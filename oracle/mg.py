"""Oracle: DD-alpha-AMG (Sec. 1.1 of arXiv:1710.06198), plain FP64.

The paper states the method through the error propagation of Eq. (1),
    eps <- (I - M D)^k (I - P D_c^-1 P^dag D) eps,
with M the SAP smoother, k smoothing iterations, P the aggregation-based
prolongation built from N_v test vectors of an adaptive setup, and the
Galerkin coarse operator D_c = P^dag D P.  P is Gamma5-compatible
(Gamma5 P = P Gamma5,c), so D_c^dag = Gamma5,c D_c Gamma5,c, and the
twisted-mass coarse operator is D_c(+-mu) = D_c +- i mu Gamma5,c with the
same P for both signs.  A flexible Krylov method (FGMRES) is preconditioned
by one application of this multigrid cycle at every step.

Details the paper leaves to its references (standard readings):
  * aggregates are lattice blocks; each test vector is split by chirality
    inside each aggregate and the pieces are orthonormalised in order by
    classical Gram-Schmidt with one re-orthogonalisation pass (positive
    real diagonal); coarse dof index = s*N_v + i, s = 0 (upper spins) / 1;
  * SAP: blocks coloured by the parity of the block-coordinate sum, colour 0
    first; each block solve is s steps of minimal residual (MR) on the
    block-restricted (Dirichlet) operator, starting from zero, with the
    block residual recomputed as r_B = eta_B - (D z)_B before each solve;
  * post-smoothing only (as Eq. (1) is written); coarse solves: GMRES on
    the coarsest level, FGMRES preconditioned by the next cycle in between;
  * setup: random test vectors, two smoother applications, then n_setup
    iterations of v_i <- B_MG v_i with P and D_c rebuilt after each.

Fields at any level: complex128 [..., T, Z, Y, X, d] with chirality halves
of the last axis.  Coarse lattices are periodic (the fine time-boundary
sign is absorbed into D_c's hopping blocks).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import torch

from .dirac import CDT, gamma5_dof, shift

# ============================================================== geometry
def coords(dims):
    """Integer coordinate arrays (x, y, z, t), each [T, Z, Y, X]."""
    lx, ly, lz, lt = dims
    t, z, y, x = torch.meshgrid(torch.arange(lt), torch.arange(lz),
                                torch.arange(ly), torch.arange(lx), indexing="ij")
    return (x, y, z, t)


def to_blocks(f: torch.Tensor, blk, split_chirality: bool) -> torch.Tensor:
    """[..., T, Z, Y, X, d] -> [..., Tc, Zc, Yc, Xc, (2,) n_loc].

    Local order inside a block: (bt, bz, by, bx, [d or d/2]) with x fastest.
    """
    bx, by, bz, bt = blk
    *lead, lt, lz, ly, lx, d = f.shape
    nb = len(lead)
    if split_chirality:
        f = f.reshape(*lead, lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx, 2, d // 2)
        perm = list(range(nb)) + [nb + i for i in (0, 2, 4, 6, 8, 1, 3, 5, 7, 9)]
        f = f.permute(perm)
        return f.reshape(*lead, lt // bt, lz // bz, ly // by, lx // bx, 2, bt * bz * by * bx * d // 2)
    f = f.reshape(*lead, lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx, d)
    perm = list(range(nb)) + [nb + i for i in (0, 2, 4, 6, 1, 3, 5, 7, 8)]
    f = f.permute(perm)
    return f.reshape(*lead, lt // bt, lz // bz, ly // by, lx // bx, bt * bz * by * bx * d)


def from_blocks(g: torch.Tensor, blk, d: int, split_chirality: bool) -> torch.Tensor:
    """Inverse of to_blocks."""
    bx, by, bz, bt = blk
    if split_chirality:
        *lead, tc, zc, yc, xc, two, n = g.shape
        nb = len(lead)
        g = g.reshape(*lead, tc, zc, yc, xc, 2, bt, bz, by, bx, d // 2)
        # current: lead, tc,zc,yc,xc, s, bt,bz,by,bx, k  -> lead, tc,bt,zc,bz,yc,by,xc,bx, s,k
        perm = list(range(nb)) + [nb + i for i in (0, 5, 1, 6, 2, 7, 3, 8, 4, 9)]
        g = g.permute(perm)
    else:
        *lead, tc, zc, yc, xc, n = g.shape
        nb = len(lead)
        g = g.reshape(*lead, tc, zc, yc, xc, bt, bz, by, bx, d)
        perm = list(range(nb)) + [nb + i for i in (0, 4, 1, 5, 2, 6, 3, 7, 8)]
        g = g.permute(perm)
    return g.reshape(*lead, tc * bt, zc * bz, yc * by, xc * bx, d)


def block_colour(dims, blk) -> torch.Tensor:
    """0/1 colour of the SAP block containing each site: [T, Z, Y, X]."""
    x = coords(dims)
    s = sum(x[m] // blk[m] for m in range(4))
    return s % 2


def check_blocking(dims, blk):
    for m in range(4):
        if dims[m] % blk[m]:
            raise ValueError(f"block {blk} does not tile lattice {dims}")
        nb = dims[m] // blk[m]
        if nb != 1 and nb % 2:
            raise ValueError(f"SAP needs an even number of blocks (or one) per dimension: {dims}/{blk}")


# ============================================================== coarse operator
class CoarseOp:
    """D_c on a periodic coarse lattice with d dof per site.

    D_c e(y) = S(y) e(y) + sum_mu [ F_mu(y) e(y+mu) + B_mu(y) e(y-mu) ] + i mu Gamma5,c e(y)
    self_blk: [T, Z, Y, X, d, d]; fwd/bwd: [4, T, Z, Y, X, d, d] (row, column).
    """

    def __init__(self, self_blk, fwd, bwd):
        self.S = self_blk
        self.F = fwd
        self.B = bwd
        lt, lz, ly, lx, d, _ = self_blk.shape
        self.dims = (lx, ly, lz, lt)
        self.dof = d
        self.g5 = gamma5_dof(d)

    def diag(self, e, mu_tm: float = 0.0):
        out = torch.einsum("...ij,...j->...i", self.S, e)
        if mu_tm != 0.0:
            out = out + 1j * mu_tm * self.g5 * e
        return out

    def hop(self, e, mu: int, direction: int):
        if direction > 0:
            return torch.einsum("...ij,...j->...i", self.F[mu], shift(e, mu, +1, xaxis=-2))
        return torch.einsum("...ij,...j->...i", self.B[mu], shift(e, mu, -1, xaxis=-2))

    def apply(self, e, mu_tm: float = 0.0):
        out = self.diag(e, mu_tm)
        for m in range(4):
            out = out + self.hop(e, m, +1) + self.hop(e, m, -1)
        return out

    def dense(self, mu_tm: float = 0.0):
        lx, ly, lz, lt = self.dims
        n = lx * ly * lz * lt * self.dof
        eye = torch.eye(n, dtype=CDT).reshape(n, lt, lz, ly, lx, self.dof)
        return self.apply(eye, mu_tm).reshape(n, n).T.contiguous()


# ============================================================== aggregation
class Prolongation:
    """P for one coarsening: orthonormal columns per (aggregate, chirality).

    Q: [Tc, Zc, Yc, Xc, 2, n_loc, Nv] with n_loc = |aggregate| * d/2.
    """

    def __init__(self, Q, agg, fine_dims, fine_dof):
        self.Q = Q
        self.agg = tuple(agg)
        self.fine_dims = tuple(fine_dims)
        self.fine_dof = fine_dof
        self.nv = Q.shape[-1]
        lx, ly, lz, lt = fine_dims
        self.coarse_dims = (lx // agg[0], ly // agg[1], lz // agg[2], lt // agg[3])

    def restrict(self, f):
        """P^dag f: r(y, s*Nv + i) = sum_{x in y, k in s} conj(v_i^{(s)}(x)_k) f(x)_k."""
        fb = to_blocks(f, self.agg, True)
        r = torch.einsum("tzyxskn,...tzyxsk->...tzyxsn", self.Q.conj(), fb)
        return r.reshape(*r.shape[:-2], 2 * self.nv)

    def prolong(self, e):
        """P e."""
        eb = e.reshape(*e.shape[:-1], 2, self.nv)
        fb = torch.einsum("tzyxskn,...tzyxsn->...tzyxsk", self.Q, eb)
        return from_blocks(fb, self.agg, self.fine_dof, True)


def block_gram_schmidt(V: torch.Tensor, agg) -> torch.Tensor:
    """Orthonormalise test vectors per aggregate and chirality.

    V: [Nv, T, Z, Y, X, d].  Classical Gram-Schmidt in index order with one
    re-orthogonalisation pass; the diagonal of R is real positive.
    Returns Q: [Tc, Zc, Yc, Xc, 2, n_loc, Nv].
    """
    vb = to_blocks(V, agg, True)               # [Nv, Tc, Zc, Yc, Xc, 2, n]
    vb = vb.movedim(0, -1).clone()             # [Tc, Zc, Yc, Xc, 2, n, Nv]
    nv = vb.shape[-1]
    for i in range(nv):
        w = vb[..., i]
        for _ in range(2):
            if i > 0:
                q = vb[..., :i]
                c = torch.einsum("...ni,...n->...i", q.conj(), w)
                w = w - torch.einsum("...ni,...i->...n", q, c)
        nrm = torch.sqrt(torch.sum((w.conj() * w).real, dim=-1, keepdim=True))
        vb[..., i] = w / nrm
    return vb


def build_prolongation(V, agg, fine_dims, fine_dof) -> Prolongation:
    return Prolongation(block_gram_schmidt(V, agg), agg, fine_dims, fine_dof)


def galerkin(op, P: Prolongation) -> CoarseOp:
    """D_c = P^dag D P, split by which fine terms connect which aggregates.

    D = diag + sum_{mu,+-} H_mu^{+-}.  A hop H_mu^+ at fine site x pulls from
    x + mu; it connects aggregate y to y + mu exactly when x sits on the
    upper face of its aggregate in direction mu (local coordinate a_mu - 1),
    and stays inside y otherwise.  For each coarse column c the prolonged
    unit field w = P e_c (column c on every aggregate) is pushed through
    each term and restricted:
        S[:, c]     = P^dag (diag w + sum of aggregate-internal hops of w)
        F_mu[:, c]  = P^dag (face-crossing H_mu^+ w)
        B_mu[:, c]  = P^dag (face-crossing H_mu^- w)
    The twisted-mass term is not included: D_c(mu) = D_c + i mu Gamma5,c.
    """
    dims, agg, d = P.fine_dims, P.agg, P.fine_dof
    x = coords(dims)
    up = [((x[m] % agg[m]) == agg[m] - 1).to(torch.float64)[..., None] for m in range(4)]
    lo = [((x[m] % agg[m]) == 0).to(torch.float64)[..., None] for m in range(4)]
    lxc, lyc, lzc, ltc = P.coarse_dims
    dc = 2 * P.nv
    S = torch.zeros(ltc, lzc, lyc, lxc, dc, dc, dtype=CDT)
    F = torch.zeros(4, ltc, lzc, lyc, lxc, dc, dc, dtype=CDT)
    B = torch.zeros(4, ltc, lzc, lyc, lxc, dc, dc, dtype=CDT)
    for c in range(dc):
        e = torch.zeros(ltc, lzc, lyc, lxc, dc, dtype=CDT)
        e[..., c] = 1.0
        w = P.prolong(e)
        s_field = op.diag(w, 0.0)
        for m in range(4):
            hp = op.hop(w, m, +1)
            hm = op.hop(w, m, -1)
            s_field = s_field + (1 - up[m]) * hp + (1 - lo[m]) * hm
            F[m, ..., c] = P.restrict(up[m] * hp)
            B[m, ..., c] = P.restrict(lo[m] * hm)
        S[..., c] = P.restrict(s_field)
    return CoarseOp(S, F, B)


# ============================================================== SAP / MR
def _block_sum(f, blk):
    """Per-SAP-block sums of a site field [..., T, Z, Y, X, d] -> broadcastable."""
    b = to_blocks(f, blk, False).sum(-1)          # [..., Tc, Zc, Yc, Xc]
    return b


def _block_expand(s, blk, like):
    """Broadcast a per-block scalar [..., Tc, Zc, Yc, Xc] back to sites [..., T, Z, Y, X, 1]."""
    bx, by, bz, bt = blk
    s = s.repeat_interleave(bt, dim=-4).repeat_interleave(bz, dim=-3)
    s = s.repeat_interleave(by, dim=-2).repeat_interleave(bx, dim=-1)
    return s[..., None]


def mr_block_solve(op, r, mask, blk, steps: int, mu_tm: float):
    """MR on every block of one colour at once (block-Dirichlet operator).

    e = 0, rho = r; repeat: q = D_B rho, alpha = <q, rho>/<q, q> per block,
    e += alpha rho, rho -= alpha q.  Returns (e, rho).
    Blocks of one colour only neighbour blocks of the other colour, so
    mask * D(mask * rho) is D_B rho on every block simultaneously.
    """
    e = torch.zeros_like(r)
    rho = r.clone()
    for _ in range(steps):
        q = mask * op.apply(mask * rho, mu_tm)
        qq = _block_sum((q.conj() * q).real, blk)
        qr = _block_sum(q.conj() * rho, blk)
        alpha = torch.where(qq > 0, qr / torch.where(qq > 0, qq, torch.ones_like(qq)),
                            torch.zeros_like(qr))
        a = _block_expand(alpha, blk, r)
        e = e + a * rho
        rho = rho - a * q
    return e, rho


def sap(op, eta, z0, mu_tm: float, blk, sweeps: int, mr_steps: int, block_solver=None):
    """k sweeps of SAP for D z = eta starting from z0 (multiplicative, 2 colours).

    block_solver(r, mask) -> e solves the block systems of one colour; the
    default is mr_steps of MR.
    """
    check_blocking(op.dims, blk)
    colour = block_colour(op.dims, blk)
    masks = [(colour == c).to(torch.float64)[..., None] for c in (0, 1)]
    z = z0.clone()
    for _ in range(sweeps):
        for c in (0, 1):
            r = masks[c] * (eta - op.apply(z, mu_tm))
            if block_solver is None:
                e, _ = mr_block_solve(op, r, masks[c], blk, mr_steps, mu_tm)
            else:
                e = block_solver(r, masks[c])
            z = z + e
    return z


# ============================================================== Krylov
@dataclass
class KrylovResult:
    x: torch.Tensor
    iters: int
    resid: List[float]          # implicit relative residual after each step
    converged: bool


def fgmres(apply_a: Callable, b: torch.Tensor, tol: float, restart: int, maxiter: int,
           apply_m: Optional[Callable] = None, x0: Optional[torch.Tensor] = None) -> KrylovResult:
    """Right-preconditioned flexible GMRES(restart) with modified Gram-Schmidt
    and Givens rotations; stops when the implicit residual <= tol*||b||.
    apply_m None means GMRES (z_j = v_j)."""
    bn = float(torch.linalg.vector_norm(b))
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    hist = []
    if bn == 0:
        return KrylovResult(torch.zeros_like(b), 0, [0.0], True)
    it = 0
    while it < maxiter:
        r = b - apply_a(x) if it > 0 or x0 is not None else b.clone()
        beta = float(torch.linalg.vector_norm(r))
        if beta <= tol * bn:
            return KrylovResult(x, it, hist, True)
        m = min(restart, maxiter - it)
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        j_done = 0
        conv = False
        for j in range(m):
            z = V[j] if apply_m is None else apply_m(V[j])
            Z.append(z)
            w = apply_a(z)
            for i in range(j + 1):
                H[i, j] = complex(torch.sum(V[i].conj() * w))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(torch.linalg.vector_norm(w))
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            a, bb = H[j, j], H[j + 1, j]
            den = math.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            # rotation [[c, s], [-conj(s), conj(c)]] with c = conj(a)/den, s = conj(b)/den
            cs[j] = np.conj(a) / den
            sn[j] = np.conj(bb) / den
            H[j, j] = den
            H[j + 1, j] = 0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) <= tol * bn:
                conv = True
                break
            if H[j, j] == 0 or float(torch.linalg.vector_norm(w)) == 0:
                conv = True
                break
            V.append(w / float(torch.linalg.vector_norm(w)))
        # the rotated Hessenberg is upper-triangular: back substitution
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:j_done], y[i + 1:j_done])) / H[i, i]
        for i in range(j_done):
            x = x + complex(y[i]) * Z[i]
        if conv:
            return KrylovResult(x, it, hist, True)
    return KrylovResult(x, it, hist, False)


# ============================================================== hierarchy
@dataclass
class MGParams:
    nlevels: int = 2
    agg: tuple = ((4, 4, 4, 4),)
    nv: tuple = (12,)
    sap_block: tuple = ((4, 4, 4, 4),)
    sap_sweeps: tuple = (4, 2)
    mr_steps: int = 4
    setup_iters: int = 3
    init_smooth: int = 2
    l2_restart: int = 10
    l2_maxiter: int = 10
    l2_tol: float = 0.1
    coarsest_tol: float = 0.1
    coarsest_maxiter: Optional[int] = None   # default: 100 (2 levels) / 50 (3 levels)

    def coarsest_iters(self):
        if self.coarsest_maxiter is not None:
            return self.coarsest_maxiter
        return 100 if self.nlevels == 2 else 50


@dataclass
class Level:
    op: object
    index: int
    P: Optional[Prolongation] = None
    tv: Optional[torch.Tensor] = None      # test vectors [Nv, T, Z, Y, X, d]
    nxt: Optional["Level"] = None


class Hierarchy:
    """The DD-alpha-AMG hierarchy and its preconditioner B_MG (Eq. (1))."""

    def __init__(self, fine_op, params: MGParams, mu_tm: float):
        self.params = params
        self.mu = mu_tm
        self.levels: List[Level] = [Level(fine_op, 0)]
        self.stats = {"coarse_iters": 0, "coarsest_iters": 0}

    # ---------------------------------------------------------- cycle
    def precondition(self, lvl: Level, v, mu_tm: float):
        """One application of Eq. (1)'s cycle: coarse correction, then k SAP sweeps."""
        p = self.params
        rc = lvl.P.restrict(v)
        ec = self.coarse_solve(lvl.nxt, rc, mu_tm)
        z = lvl.P.prolong(ec)
        return sap(lvl.op, v, z, mu_tm, p.sap_block[lvl.index],
                   p.sap_sweeps[lvl.index], p.mr_steps)

    def coarse_solve(self, lvl: Level, rc, mu_tm: float):
        p = self.params
        a = lambda e: lvl.op.apply(e, mu_tm)
        if lvl.nxt is None:
            res = fgmres(a, rc, p.coarsest_tol, p.coarsest_iters(), p.coarsest_iters())
            self.stats["coarsest_iters"] += res.iters
            return res.x
        m = lambda v: self.precondition(lvl, v, mu_tm)
        res = fgmres(a, rc, p.l2_tol, p.l2_restart, p.l2_maxiter, apply_m=m)
        self.stats["coarse_iters"] += res.iters
        return res.x

    # ---------------------------------------------------------- setup
    def _smooth_vectors(self, lvl: Level, V):
        p = self.params
        out = []
        for i in range(V.shape[0]):
            v = V[i]
            for _ in range(p.init_smooth):
                v = sap(lvl.op, v, torch.zeros_like(v), self.mu, p.sap_block[lvl.index],
                        p.sap_sweeps[lvl.index], p.mr_steps)
                v = v / torch.linalg.vector_norm(v)
            out.append(v)
        return torch.stack(out)

    def _build_next(self, lvl: Level):
        p = self.params
        lvl.P = build_prolongation(lvl.tv, p.agg[lvl.index], lvl.op.dims, lvl.op.dof)
        dc = galerkin(lvl.op, lvl.P)
        if lvl.nxt is None:
            lvl.nxt = Level(dc, lvl.index + 1)
        else:
            lvl.nxt.op = dc

    def setup(self, test_vectors: List[torch.Tensor]):
        """Adaptive setup: test_vectors[l] are the random start vectors of level l.

        Initial phase: v_i <- SAP(v_i) twice (normalised), then P and D_c;
        then setup_iters iterations of v_i <- B_MG v_i and a rebuild.
        """
        p = self.params
        lvl = self.levels[0]
        for li in range(p.nlevels - 1):
            lvl.tv = self._smooth_vectors(lvl, torch.as_tensor(test_vectors[li], dtype=CDT))
            self._build_next(lvl)
            if li + 1 < p.nlevels - 1:
                self.levels.append(lvl.nxt)
            lvl = lvl.nxt
        for _ in range(p.setup_iters):
            self.setup_iteration()

    def setup_iteration(self):
        """v_i <- B_MG v_i on each level in turn, rebuilding P and D_c after each.

        When a level below the rebuilt coarse operator exists, its Galerkin
        operator is rebuilt at once from its current P, so that the cycle
        used to update the next level's vectors is consistent.
        """
        p = self.params
        for li in range(p.nlevels - 1):
            lvl = self.levels[li]
            new = []
            for i in range(lvl.tv.shape[0]):
                v = self.precondition(lvl, lvl.tv[i], self.mu)
                new.append(v / torch.linalg.vector_norm(v))
            lvl.tv = torch.stack(new)
            self._build_next(lvl)
            if lvl.nxt.nxt is not None:
                self._build_next(lvl.nxt)

    # ---------------------------------------------------------- solve
    def solve(self, b, tol: float, restart: int = 30, maxiter: int = 1000, mu_tm=None):
        mu_tm = self.mu if mu_tm is None else mu_tm
        fine = self.levels[0]
        a = lambda v: fine.op.apply(v, mu_tm)
        m = lambda v: self.precondition(fine, v, mu_tm)
        return fgmres(a, b, tol, restart, maxiter, apply_m=m)


def random_test_vectors(dims, dof: int, nv: int, seed: int) -> torch.Tensor:
    """Complex Gaussian start vectors [Nv, T, Z, Y, X, dof] (Re, Im ~ N(0, 1/2))."""
    from lattice_inputs import gaussian_spinor
    v = gaussian_spinor(dims, seed, n=nv, dof=(dof,))
    return torch.as_tensor(v, dtype=CDT)


def setup_vectors(params: MGParams, fine_dims, seed: int):
    """Start vectors for every coarsening (level 0 fine, level 1 coarse, ...)."""
    out = []
    dims, dof = tuple(fine_dims), 12
    for li in range(params.nlevels - 1):
        out.append(random_test_vectors(dims, dof, params.nv[li], seed + 100 * li))
        a = params.agg[li]
        dims = tuple(dims[m] // a[m] for m in range(4))
        dof = 2 * params.nv[li]
    return out


# ============================================================== drivers
def two_step_solve(hier: Hierarchy, b, mu_tm: float, tol: float, **kw):
    """D(mu)^dag D(mu) y = b in two steps with one hierarchy (Sec. 1.1):
    D(-mu) x = Gamma5 b, then D(mu) y = Gamma5 x."""
    g5 = hier.levels[0].op.g5
    x = hier.solve(g5 * b, tol, mu_tm=-mu_tm, **kw).x
    return hier.solve(g5 * x, tol, mu_tm=mu_tm, **kw).x


def shifted_solve(hier: Hierarchy, b, sigma: float, mu_tm: float, tol: float, **kw):
    """(D D^dag + sigma) x = b.

    D(mu) D(mu)^dag = Gamma5 (Q^2 + mu^2) Gamma5 with Q = Gamma5 D(0)
    Hermitian, so D D^dag + sigma = D(mu') D(mu')^dag, mu' = sqrt(mu^2 + sigma).
    Solve D(mu') w = b, then D(mu')^dag x = w, i.e. x = Gamma5 D(-mu')^-1 Gamma5 w.
    """
    mup = math.sqrt(mu_tm * mu_tm + sigma)
    g5 = hier.levels[0].op.g5
    w = hier.solve(b, tol, mu_tm=mup, **kw).x
    u = hier.solve(g5 * w, tol, mu_tm=-mup, **kw).x
    return g5 * u
