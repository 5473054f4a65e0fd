"""Seeded synthetic inputs and workload definitions (no solver arithmetic)."""
from .gen import *  # noqa: F401,F403
from .configs import WORKLOADS, Workload, workload, load_m0  # noqa: F401
