"""Spherical (Michel) accretion onto a Schwarzschild black hole (M = 1).

The stationary solution the paper's regression tests keep (Readiness and
Testing section: Bondi accretion with its convergence), written out here
independently of the scheme, as point values at zone centres of a modified
Kerr-Schild grid with a = 0:

* polytrope p = K rho^gamma, u = p/(gamma - 1), Theta = p/rho, specific
  enthalpy h = 1 + gamma/(gamma - 1) Theta;
* mass flux 4 pi r^2 rho u^r = -mdot and Bernoulli h^2 (1 - 2/r + (u^r)^2) =
  const are conserved along r;
* at the sonic radius r_c: (u^r)^2 = 1/(2 r_c) and the sound speed
  c_s^2 = gamma Theta / h equals (u^r)^2 / (1 - 3 (u^r)^2) (Michel 1972),
  which fixes Theta_c, K (given rho_c) and the two constants;
* at every other radius rho solves the Bernoulli relation on the
  supersonic branch inside r_c and the subsonic branch outside;
* u^t follows from u.u = -1 in Kerr-Schild coordinates, (z u^r +
  sqrt(1 - z + (u^r)^2)) / (1 - z) with z = 2/r (Schwarzschild u^t plus
  2/(r - 2) u^r); in the modified coordinates u^1 = u^r / r and
  u~^1 = u^1 - u^t g^{t1}/g^{tt}.

Ghost zones carry the same solution (frozen radial boundaries); x2 has the
polar boundaries, x3 one periodic zone.  B = 0.
"""

import math
import numpy as np

from .spec import GridSpec, NG, NVAR, BC_FROZEN, BC_POLAR, BC_PERIODIC, METRIC_KERR_MKS


def michel_constants(rc=8.0, gamma=4.0 / 3.0, rho_c=1.0):
    urc2 = 1.0 / (2.0 * rc)
    cs2 = urc2 / (1.0 - 3.0 * urc2)
    n = gamma / (gamma - 1.0)
    theta_c = cs2 / (gamma - n * cs2)          # cs2 = gamma Theta / (1 + n Theta)
    K = theta_c / rho_c ** (gamma - 1.0)
    mdot = 4.0 * math.pi * rc * rc * rho_c * math.sqrt(urc2)
    hc = 1.0 + n * theta_c
    bern = hc * hc * (1.0 - 2.0 / rc + urc2)
    return dict(rc=rc, gamma=gamma, K=K, mdot=mdot, bern=bern, rho_c=rho_c)


def _residual(rho, r, c):
    g = c["gamma"]
    theta = c["K"] * rho ** (g - 1.0)
    h = 1.0 + g / (g - 1.0) * theta
    ur = c["mdot"] / (4.0 * math.pi * r * r * rho)
    return h * h * (1.0 - 2.0 / r + ur * ur) / c["bern"] - 1.0


def michel_rho(r, c):
    """Density at radius r: minimise the Bernoulli residual in log rho (its
    one minimum separates the two branches), then bisect on the branch."""
    f = lambda lr: _residual(math.exp(lr), r, c)
    lo, hi = math.log(c["rho_c"]) - 40.0, math.log(c["rho_c"]) + 40.0
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    for _ in range(200):
        x1 = b - gr * (b - a)
        x2 = a + gr * (b - a)
        if f(x1) < f(x2):
            b = x2
        else:
            a = x1
    lmin = 0.5 * (a + b)
    if abs(r - c["rc"]) < 1e-12:
        return math.exp(lmin)
    # supersonic (low density) inside the sonic radius, subsonic outside
    a, b = (lo, lmin) if r < c["rc"] else (lmin, hi)
    fa = f(a)
    for _ in range(200):
        m = 0.5 * (a + b)
        fm = f(m)
        if (fm > 0.0) == (fa > 0.0):
            a, fa = m, fm
        else:
            b = m
    return math.exp(0.5 * (a + b))


def bondi_grid(n1, n2, n3=1, rin=1.9, rout=20.0, hslope=1.0):
    return GridSpec(n1, n2, n3,
                    x1min=math.log(rin), x1max=math.log(rout),
                    x2min=0.0, x2max=1.0, x3min=0.0, x3max=2.0 * math.pi,
                    bc=(BC_FROZEN, BC_FROZEN, BC_POLAR, BC_POLAR, BC_PERIODIC, BC_PERIODIC),
                    metric=METRIC_KERR_MKS, a=0.0, hslope=hslope)


def bondi(n1, n2, n3=1, rc=8.0, gamma=4.0 / 3.0, rin=1.9, rout=20.0, hslope=1.0):
    """Grid, padded prims of the Michel flow and its constants."""
    grid = bondi_grid(n1, n2, n3, rin=rin, rout=rout, hslope=hslope)
    c = michel_constants(rc=rc, gamma=gamma)
    x1, _, _ = grid.centers()
    r = np.exp(x1)
    rho = np.array([michel_rho(float(ri), c) for ri in r])
    ur = -c["mdot"] / (4.0 * math.pi * r * r * rho)
    u = c["K"] * rho ** gamma / (gamma - 1.0)
    # Kerr-Schild u^t from u.u = -1 (future root; the same expression as the
    # Schwarzschild u^t plus 2/(r - 2) u^r, regular through the horizon)
    z = 2.0 / r
    f = 1.0 - z
    ut = (z * ur + np.sqrt(f + ur * ur)) / f
    u1 = ur / r
    gtt_con = -(1.0 + z)                        # KS g^{tt} (a = 0)
    gt1_con = z / r                             # KS g^{tr} / r
    ut1 = u1 - ut * gt1_con / gtt_con
    P = np.zeros((NVAR, n3 + 2 * NG, n2 + 2 * NG, n1 + 2 * NG))
    P[0] = rho[None, None, :]
    P[1] = u[None, None, :]
    P[2] = ut1[None, None, :]
    return grid, P, c
