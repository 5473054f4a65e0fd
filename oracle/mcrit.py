"""Oracle: the bare mass m0 of a synthetic workload.

The workloads fix m0 as minus the smallest real part of the spectrum of the
clover-improved Wilson operator at m0 = 0, mu = 0, plus 0.005.  The literal
"smallest real eigenvalue" is ill-posed (the free operator with an even
time extent has no real eigenvalue), so the eigenvalue with the smallest
real part is used; ARPACK (scipy.sparse.linalg.eigs, which='SR') finds it.

Only the 8^4 workload states this recipe for its own lattice.  For the
larger workloads (which give no m0) the same recipe is applied to an 8^4
lattice drawn with the workload's link spread, c_sw and link seed: the
critical mass is an intensive quantity, and ARPACK at their full volumes
would take hours on the host.  With mu > 0 the operator stays invertible
(D D^dag >= mu^2) even if the full volume holds a slightly lower mode.

Run as a script to write lattice_inputs/m0.json:
    python -m oracle.mcrit c1 c4 c2 ...
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import torch
from scipy.sparse.linalg import LinearOperator, eigs

from .dirac import WilsonClover


def smallest_real_part(U, csw: float, ncv: int = 64, tol: float = 1e-8, k: int = 4):
    """Eigenvalue of D(m0 = 0, mu = 0) with the smallest real part."""
    op = WilsonClover(U, 0.0, csw)
    lx, ly, lz, lt = op.dims
    n = lx * ly * lz * lt * 12

    def mv(v):
        f = torch.as_tensor(np.asarray(v).reshape(lt, lz, ly, lx, 12), dtype=torch.complex128)
        return op.apply(f, 0.0).reshape(-1).numpy()

    lin = LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    rng = np.random.default_rng(12345)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    w = eigs(lin, k=k, which="SR", ncv=min(ncv, n - 2), tol=tol, v0=v0,
             return_eigenvectors=False, maxiter=100000)
    return w[np.argmin(w.real)]


PROXY_DIMS = (8, 8, 8, 8)


def m0_for(name: str, **kw):
    from lattice_inputs import workload, gauge_links
    w = workload(name)
    dims = tuple(w.dims) if w.volume <= 8 ** 4 else PROXY_DIMS
    U = gauge_links(dims, w.eps, w.seeds["links"])
    lam = smallest_real_part(U, w.csw, **kw)
    m0 = -float(lam.real) + 0.005
    return {"m0": m0, "kappa": 1.0 / (2 * m0 + 8), "eig_dims": list(dims),
            "lambda_sr": [float(lam.real), float(lam.imag)]}


def main(names):
    from lattice_inputs.configs import m0_path
    path = m0_path()
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    for nm in names:
        t0 = time.time()
        r = m0_for(nm)
        r["seconds"] = round(time.time() - t0, 1)
        r["threads"] = torch.get_num_threads()
        data[nm] = r
        print(nm, r, flush=True)
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
