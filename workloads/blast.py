"""Cylindrical explosion in a strongly magnetised medium (flat space).

A standard stress test of relativistic MHD codes (Komissarov 1999): on the
periodic square [-6, 6]^2 (one zone, or a few, along x3) gas at rest with
rho = 1e-2, p = 1 inside r < r_in = 0.8 and rho = 1e-4, p = 3e-5 outside
r_out = 1, joined linearly in log rho and log p between, threaded by a
uniform field B^1 = B0 (the default 0.07 gives b^2/rho = 49 in the ambient
gas and beta = 2 p/b^2 = 1.2e-2; Komissarov's weak-field case has 0.1).  The explosion drives a fast shock into gas whose
magnetisation the high-order scheme cannot resolve, which is what the
first-order flux correction and the floors are for.  gamma = 4/3; u = p/(gamma - 1).
A seeded relative perturbation of the inner pressure (amplitude `noise`)
breaks the grid symmetry when asked for.
"""

import math

import numpy as np

from .spec import GridSpec, NG, NVAR, BC_PERIODIC, METRIC_MINKOWSKI


def blast_grid(n, n3=1, half=6.0):
    return GridSpec(n, n, n3, x1min=-half, x1max=half, x2min=-half, x2max=half,
                    x3min=0.0, x3max=2.0 * half * n3 / n,
                    bc=(BC_PERIODIC,) * 6, metric=METRIC_MINKOWSKI)


def magnetised_blast(n, n3=1, B0=0.07, gamma=4.0 / 3.0, r_in=0.8, r_out=1.0,
                     rho_in=1e-2, p_in=1.0, rho_out=1e-4, p_out=3e-5, noise=0.0, seed=0,
                     faces=False):
    """Grid and padded prims of the explosion (and, with faces, the face
    fields of face-centred constrained transport: B0 on every x1 face)."""
    grid = blast_grid(n, n3)
    x1, x2, _ = grid.centers()
    X, Y = np.meshgrid(x1, x2, indexing="xy")          # (n2+2g, n1+2g)
    r = np.sqrt(X * X + Y * Y)
    s = np.clip((r - r_in) / (r_out - r_in), 0.0, 1.0)
    rho = np.exp((1 - s) * math.log(rho_in) + s * math.log(rho_out))
    p = np.exp((1 - s) * math.log(p_in) + s * math.log(p_out))
    shape = (n3 + 2 * NG,) + X.shape
    P = np.zeros((NVAR,) + shape)
    P[0] = rho[None]
    P[1] = p[None] / (gamma - 1.0)
    if noise:
        rng = np.random.default_rng(seed)
        P[1] *= 1.0 + noise * rng.uniform(-1, 1, shape) * (r < r_in)[None]
    P[5] = B0
    if faces:
        Bf = np.zeros((3,) + shape)
        Bf[0] = B0
        return grid, P, Bf
    return grid, P
