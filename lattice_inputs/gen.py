"""Seeded synthetic inputs for the twisted-mass clover Wilson solver.

This module only draws random numbers and shapes them into gauge links,
spinor sources and test directions.  It holds none of the solver's
arithmetic; both the CPU oracle and the GPU tests/benchmark take their
inputs from here so that the two sides see identical data.

Layouts (canonical, shared with the C ABI):
  site index        = ((t*Lz + z)*Ly + y)*Lx + x   (x fastest)
  gauge links       complex128 [4][T][Z][Y][X][3][3], mu = 0..3 <-> x,y,z,t
  spinor fields     complex128 [n][T][Z][Y][X][4][3]

The paper's gauge ensembles (64^3 x 128, twisted mass at maximal twist)
are not available; random SU(3) links near unity with a tunable spread
stand in for them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "gauge_links",
    "gaussian_spinor",
    "point_sources",
    "rational_shifts",
    "su3_algebra_coeffs",
    "su3_from_coeffs",
    "random_gauge_transform",
    "md_step_links",
    "unit_links",
    "su3_momenta",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a (tr lambda_a lambda_b = 2 delta_ab)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a batch of Hermitian 3x3 matrices via eigendecomposition."""
    w, v = np.linalg.eigh(h)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Project onto SU(3): Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.cross(r0, r1).conj()
    return np.stack([r0, r1, r2], axis=-2)


def _slice_rngs(seed: int, lt: int):
    """One PCG64 stream per time slice so any t-slab can be regenerated alone."""
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(seed).spawn(lt)]


def su3_from_coeffs(coeffs: np.ndarray, scale: float) -> np.ndarray:
    """exp(i*scale*sum_a c_a lambda_a/2), re-unitarised; coeffs [..., 8]."""
    lam = gell_mann()
    h = scale * np.einsum("...a,aij->...ij", coeffs, lam) / 2
    return _reunitarise(_expi_hermitian(h))


def _links_slice(args):
    """Links of time slice t: [4][Z][Y][X][3][3] from that slice's stream."""
    dims, eps, seq, t = args
    lx, ly, lz, _ = dims
    g = np.random.Generator(np.random.PCG64(seq)).standard_normal((lz, ly, lx, 4, 8))
    return t, np.moveaxis(su3_from_coeffs(g, eps), 3, 0)


def gauge_links(dims, eps: float, seed: int, t_range=None, workers: int = 1) -> np.ndarray:
    """Random links U = exp(i eps sum_a g_a lambda_a / 2), g_a ~ N(0,1).

    dims = (Lx, Ly, Lz, Lt).  Draw order: t-slice major (one stream per
    slice), then z, y, x, then mu, then a.  t_range = (t0, t1) draws only
    slices t0 <= t < t1 (the same values as in the whole field; t may run
    past Lt, wrapping); workers > 1 draws slices in that many processes
    (identical result).
    Returns complex128 [4][T][Z][Y][X][3][3] (T = t1 - t0 with t_range).
    """
    lx, ly, lz, lt = dims
    t0, t1 = (0, lt) if t_range is None else t_range
    seqs = np.random.SeedSequence(seed).spawn(lt)
    jobs = [(dims, eps, seqs[t % lt], t - t0) for t in range(t0, t1)]
    out = np.empty((4, t1 - t0, lz, ly, lx, 3, 3), dtype=np.complex128)
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            for t, u in pool.imap_unordered(_links_slice, jobs):
                out[:, t] = u
    else:
        for job in jobs:
            t, u = _links_slice(job)
            out[:, t] = u
    return out


def unit_links(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def gaussian_spinor(dims, seed: int, n: int = 1, dof=(4, 3)) -> np.ndarray:
    """Complex Gaussian field, Re and Im ~ N(0, 1/2) so E|z|^2 = 1.

    Returns complex128 [n][T][Z][Y][X][*dof].
    """
    lx, ly, lz, lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n, lt, lz, ly, lx) + tuple(dof)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def point_sources(dims, seed: int, n: int = 12) -> np.ndarray:
    """n spin-colour point sources; source k sits at its own random site,
    spin k//3, colour k%3, value 1.  Returns [n][T][Z][Y][X][4][3]."""
    lx, ly, lz, lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((n, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
    for k in range(n):
        x, y, z, t = (int(rng.integers(0, l)) for l in (lx, ly, lz, lt))
        out[k, t, z, y, x, (k // 3) % 4, k % 3] = 1.0
    return out


def rational_shifts(n: int = 8, lo_exp: float = -5.0, hi_exp: float = 0.0) -> np.ndarray:
    """n shifts sigma_k log-spaced in [10^lo_exp, 10^hi_exp]."""
    k = np.arange(n)
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * k / (n - 1))


def su3_algebra_coeffs(dims, seed: int) -> np.ndarray:
    """omega^a_mu(x) ~ N(0,1), i.i.d. over links: float64 [4][T][Z][Y][X][8]."""
    lx, ly, lz, lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((4, lt, lz, ly, lx, 8))


def md_step_links(U: np.ndarray, step: float, seed: int) -> np.ndarray:
    """One step of a random walk on the links, a stand-in for a molecular
    dynamics update: U'_mu(x) = exp(i step sum_a g_a lambda_a / 2) U_mu(x),
    g_a ~ N(0,1) i.i.d. per link.  U: complex128 [4][T][Z][Y][X][3][3]."""
    g = np.random.Generator(np.random.PCG64(seed)).standard_normal(U.shape[:-2] + (8,))
    return _reunitarise(np.matmul(su3_from_coeffs(g, step), U))


def random_gauge_transform(dims, seed: int, scale: float = 1.0) -> np.ndarray:
    """Random SU(3) matrix per site: complex128 [T][Z][Y][X][3][3]."""
    lx, ly, lz, lt = dims
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((lt, lz, ly, lx, 8))
    return su3_from_coeffs(g, scale)


def su3_momenta(dims, seed: int) -> np.ndarray:
    """Molecular-dynamics momenta P = sum_a p^a T^a, T^a = i lambda^a / 2,
    p^a ~ N(0, 1) i.i.d. per link: complex128 [4][T][Z][Y][X][3][3]
    (traceless anti-Hermitian; the density exp(-sum |P_ij|^2) of the
    kinetic term K = sum_a (p^a)^2 / 2)."""
    c = su3_algebra_coeffs(dims, seed)
    return np.einsum("...a,aij->...ij", c, 0.5j * gell_mann())
