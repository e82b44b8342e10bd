"""Seeded synthetic inputs shared by the oracle and the device solver.

Holds the counter-based generator (``rng``), the grid/coefficient laws
(``grids``) and the workload builders (``configs``); the device generator that
reproduces them bit-for-bit is ``devgen.hip`` (``device.py`` loads it).  No
tridiagonal-solver arithmetic lives in this package.
"""
from . import rng, grids, configs  # noqa: F401
