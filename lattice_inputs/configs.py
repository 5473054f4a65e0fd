"""Workload definitions (lattice, operator parameters, solver hierarchy).

Five synthetic workloads stand in for the paper's 64^3 x 128 ensembles:
  c1  8^4       plain FP64, 2-level, single RHS (CPU-sized)
  c2  24^3x48   mixed precision, 3-level, single RHS
  c3  32^3x64   batched: 12 point sources + 8 shifted systems
  c4  16^3x32   fermion force
  c5  64^3x128  the paper's volume, all forms combined

The bare mass m0 of each workload is a stored input: it was computed by
oracle/mcrit.py (smallest-real-part eigenvalue of the clover operator at
m0 = 0, mu = 0, plus 0.005) and written to m0.json next to this file.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field, asdict

_HERE = os.path.dirname(os.path.abspath(__file__))


@dataclass
class Workload:
    name: str
    dims: tuple            # (Lx, Ly, Lz, Lt)
    eps: float             # link spread
    csw: float
    mu: float
    nlevels: int
    agg: tuple             # aggregate shape per coarsening, ((ax,ay,az,at), ...)
    nv: tuple              # test vectors per coarsening
    sap_block: tuple       # SAP block shape per smoothed level
    setup_iters: int = 3
    init_smooth: int = 2
    sap_sweeps: tuple = (4, 2)     # k on level 1, level 2
    mr_steps: int = 4
    restart: int = 30
    tol: float = 1e-10
    seed_id: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def volume(self):
        v = 1
        for d in self.dims:
            v *= d
        return v

    @property
    def seeds(self):
        c = self.seed_id
        return {"links": 1000 + c, "source": 2000 + c, "xi": 3000 + c,
                "testvec": 4000 + c, "fd": 5000 + c}

    def m0(self):
        return load_m0().get(self.name)

    def kappa(self):
        m0 = self.m0()
        return None if m0 is None else 1.0 / (2.0 * m0 + 8.0)

    def to_dict(self):
        return asdict(self)


WORKLOADS = {
    "c1": Workload("c1", (8, 8, 8, 8), 0.3, 1.0, 0.01, 2,
                   ((4, 4, 4, 4),), (12,), ((4, 4, 4, 4),), seed_id=1),
    "c2": Workload("c2", (24, 24, 24, 48), 0.25, 1.6, 0.0015, 3,
                   ((4, 4, 4, 4), (2, 2, 2, 2)), (24, 32),
                   ((4, 4, 4, 4), (3, 3, 3, 3)), seed_id=2),
    "c3": Workload("c3", (32, 32, 32, 64), 0.25, 1.6, 0.0015, 3,
                   ((4, 4, 4, 4), (2, 2, 2, 2)), (24, 32),
                   ((4, 4, 4, 4), (2, 2, 2, 2)), seed_id=3,
                   extra={"n_point": 12, "n_shift": 8}),
    "c4": Workload("c4", (16, 16, 16, 32), 0.3, 1.6, 0.003, 3,
                   ((4, 4, 4, 4), (2, 2, 2, 2)), (24, 32),
                   ((4, 4, 4, 4), (2, 2, 2, 2)), seed_id=4,
                   extra={"fd_dirs": 16, "fd_h": 1e-5}),
    "c5": Workload("c5", (64, 64, 64, 128), 0.2, 1.57, 0.00072, 3,
                   ((4, 4, 4, 4), (2, 2, 2, 2)), (24, 32),
                   ((4, 4, 4, 4), (2, 2, 2, 2)), seed_id=5,
                   extra={"nrhs": 4}),
}


def m0_path():
    return os.path.join(_HERE, "m0.json")


def load_m0():
    p = m0_path()
    if not os.path.exists(p):
        return {}
    with open(p) as f:
        d = json.load(f)
    return {k: v["m0"] for k, v in d.items()}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
