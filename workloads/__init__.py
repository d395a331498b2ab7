"""Seeded synthetic inputs (meshes, grids, PSFs, arrival traces).

Shared by the tests, the benchmark and the oracle's checks.  It holds no part
of the rendering arithmetic, so neither side can borrow the other's math
through it.
"""
from . import meshes, configs  # noqa: F401
from .configs import VOLUME, SURFACE, Grid, Case, psf_diag  # noqa: F401
