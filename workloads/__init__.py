"""Seeded synthetic inputs for the HARM step: problem set-ups only.

This package builds initial primitive states and grid descriptions that the
CPU oracle and the HIP library both consume.  It holds none of the numerical
scheme (no reconstruction, Riemann solver, constrained transport, update or
inversion); the few metric and four-velocity formulas that initial data need
are written here independently of both implementations.

State layout used everywhere: float64 array of shape (8, n3+2g, n2+2g, n1+2g),
x1 fastest, variables (rho, u, u~1, u~2, u~3, B1, B2, B3), ghost width g = 3.
"""

from .spec import (NG, NVAR, BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_FROZEN,
                   METRIC_MINKOWSKI, METRIC_KERR_MKS, RECON_MC, RECON_WENO5,
                   GridSpec, padded_shape, interior)
from .linear_modes import linear_mode, linear_mode_faces, mode_eigensystem, MODES
from .torus import fm_torus, torus_grid
from .packs import torus_pack, torus_tiling, tiling
from .bondi import bondi, michel_constants, michel_rho
from .blast import magnetised_blast, blast_grid

__all__ = [
    "NG", "NVAR", "BC_PERIODIC", "BC_OUTFLOW", "BC_POLAR", "BC_FROZEN",
    "METRIC_MINKOWSKI", "METRIC_KERR_MKS", "RECON_MC", "RECON_WENO5",
    "GridSpec", "padded_shape", "interior", "linear_mode", "linear_mode_faces", "mode_eigensystem",
    "MODES", "fm_torus", "torus_grid", "torus_pack", "torus_tiling", "tiling", "bondi", "michel_constants", "michel_rho",
    "magnetised_blast", "blast_grid",
]
