"""Plain descriptions of a grid and of the padded state layout."""

from dataclasses import dataclass, field
import math

NG = 3          # ghost zones per side (enough for the 5-point WENO stencil)
NVAR = 8        # rho, u, u~1, u~2, u~3, B1, B2, B3

BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_FROZEN = 0, 1, 2, 3
METRIC_MINKOWSKI, METRIC_KERR_MKS = 0, 1
RECON_MC, RECON_WENO5 = 0, 1


@dataclass
class GridSpec:
    """Interior zone counts, coordinate extents, boundary kinds and metric.

    bc is ordered (x1-, x1+, x2-, x2+, x3-, x3+).  For the Kerr metric the
    coordinates are modified Kerr-Schild (r = exp(x1), theta from x2 with
    the hslope squeeze, phi = x3), black-hole mass 1.
    """
    n1: int
    n2: int
    n3: int
    x1min: float = 0.0
    x1max: float = 1.0
    x2min: float = 0.0
    x2max: float = 1.0
    x3min: float = 0.0
    x3max: float = 1.0
    bc: tuple = (BC_PERIODIC,) * 6
    metric: int = METRIC_MINKOWSKI
    a: float = 0.0
    hslope: float = 0.3

    @property
    def dx(self):
        return ((self.x1max - self.x1min) / self.n1,
                (self.x2max - self.x2min) / self.n2,
                (self.x3max - self.x3min) / self.n3)

    @property
    def nzones(self):
        return self.n1 * self.n2 * self.n3

    def centers(self):
        """Zone-centre coordinates (x1, x2, x3) of the padded grid, 1-D each."""
        import numpy as np
        d1, d2, d3 = self.dx
        x1 = self.x1min + (np.arange(-NG, self.n1 + NG) + 0.5) * d1
        x2 = self.x2min + (np.arange(-NG, self.n2 + NG) + 0.5) * d2
        x3 = self.x3min + (np.arange(-NG, self.n3 + NG) + 0.5) * d3
        return x1, x2, x3


def padded_shape(g: GridSpec):
    return (NVAR, g.n3 + 2 * NG, g.n2 + 2 * NG, g.n1 + 2 * NG)


def interior(a, ng=NG):
    """View of the interior zones of a padded (..., k, j, i) array."""
    return a[..., ng:-ng, ng:-ng, ng:-ng]
