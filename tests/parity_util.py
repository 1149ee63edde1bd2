"""The parity metrics shared by the GPU tests.

rel_l1: relative L1 over interior zones, per primitive: the scalars rho and
u against their own L1 norm; each component of the vectors u~ and B against
the L1 norm of the whole vector (the sum over its three components), so that
a component that vanishes in the exact solution (u~2 of an axisymmetric
torus, u~3 and B3 of a wave in the x1-x2 plane) is measured against the
field's scale and not against its own roundoff.  The bar is TOL = 1e-12 per
step for every primitive.

One exception, measured rather than assumed: a linear mode at rest has no
background velocity, so its whole u~ vector is the 1e-4 perturbation, moved
by differences of O(1) background fluxes; any change of rounding (fused
multiply-adds, a reciprocal for a quotient) shows there at ~1e-12 of the
perturbation.  Those components (NOISY_MODE) are held to NOISE_FACTOR times
the distance between the oracle and the oracle built with FMA contraction
(oracle.run(..., fma=True)) on the same case, when that exceeds TOL.

zone_rel: the largest per-zone relative difference of each primitive, the
zone's own scale being |rho|, |u|, or the sum of |components| of its vector,
plus ZONE_FLOOR of that scale's largest value over the grid (1e-10 for rho
and u; 1e-6 for the vectors, whose components where the velocity or field is
below a millionth of its largest value are rounding noise of the stronger
flow around them: the velocity outside a blast, a linear mode's u~).  It sees errors
confined to a few zones, which the L1 norm, dominated by the torus body,
does not.  The bars ZONE_TOL sit well above the oracle's own FMA spread
measured on the torus workloads (rho <= 2.5e-13; u <= 1e-9, where u << rho
in the outer atmosphere and u = (W/gamma^2 - rho)/gam cancels; vector
components <= 6e-12) and above the per-zone effect of a limiter taking the
other branch under a different rounding; where the FMA oracle's result is
at hand (alt), a bar is raised to ZONE_FACTOR times its per-zone spread:
fields that are nearly zero over part of the grid (the velocity outside a
blast, the u~ of a linear mode at rest) are rounding noise there.  An O(1)
error in any zone is 1e8 times these bars or more.
"""

import numpy as np

from workloads import interior

GROUPS = [[0], [1], [2, 3, 4], [2, 3, 4], [2, 3, 4], [5, 6, 7], [5, 6, 7], [5, 6, 7]]
TOL = 1e-12
NOISY_MODE = (2, 3, 4)
NOISE_FACTOR = 3.0
ZONE_TOL = np.array([1e-10, 1e-8, 1e-8, 1e-8, 1e-8, 1e-8, 1e-8, 1e-8])
ZONE_FLOOR = np.array([1e-10, 1e-10, 1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-6])
ZONE_FACTOR = 10.0


def rel_l1(a, b):
    A, B = interior(a), interior(b)
    out = []
    for v in range(A.shape[0]):
        den = sum(np.abs(B[w]).sum() for w in GROUPS[v])
        num = np.abs(A[v] - B[v]).sum()
        out.append(0.0 if num == 0.0 else (num / den if den > 0.0 else np.inf))
    return np.array(out)


def zone_rel(a, b, floor=ZONE_FLOOR):
    A, B = interior(a), interior(b)
    out = []
    for v in range(A.shape[0]):
        sc = sum(np.abs(B[w]) for w in GROUPS[v])
        sc = sc + floor[v] * sc.max()
        d = np.abs(A[v] - B[v])
        out.append(0.0 if not d.any() else float((d / np.where(sc > 0.0, sc, 1.0)).max()))
    return np.array(out)


def bars(noisy=(), spread=None, tol=TOL):
    """Per-primitive L1 bars: tol, or for the noisy components the larger of
    tol and NOISE_FACTOR times the oracle's FMA spread."""
    b = np.full(8, tol)
    for v in noisy:
        b[v] = max(tol, NOISE_FACTOR * spread[v])
    return b


def check(out, ref, noisy=(), spread=None, tol=TOL, zone=True, label="", alt=None):
    """Assert the L1 bars and (zone=True) the per-zone bars; alt: the FMA
    oracle's result on the same case (gives spread when it is not passed,
    and raises the per-zone bars to its per-zone spread).  Returns (rel L1,
    per-zone)."""
    if alt is not None and spread is None:
        spread = rel_l1(alt, ref)
    r = rel_l1(out, ref)
    b = bars(noisy, spread, tol)
    z = zone_rel(out, ref)
    zb = ZONE_TOL.copy()
    if alt is not None:
        zb = np.maximum(zb, ZONE_FACTOR * zone_rel(alt, ref))
    print(label, "rel L1", r, "bars", b, "per zone", z, "zone bars", zb, flush=True)
    assert np.all(r <= b), (r, b)
    if zone:
        assert np.all(z <= zb), (z, zb)
    return r, z
