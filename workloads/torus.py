"""Magnetised Fishbone-Moncrief torus around a Kerr black hole (M = 1).

Initial data for the torus accretion workload the paper times (Performance
section): ideal GRMHD in spherical (modified Kerr-Schild) coordinates.  The
construction follows the physics of a constant-l torus; every metric formula
used here is written out in this file, independently of the scheme.

* l = u^t u_phi equals its value on the prograde circular geodesic at r_max
  (Bardeen-Press-Teukolsky energy and angular momentum, Boyer-Lindquist).
* ln h(r, theta) is the Fishbone-Moncrief enthalpy relative to (r_in, pi/2);
  inside (h > 1, r >= r_in) rho = [(h-1)(g-1)/g]^(1/(g-1)) normalised to a
  maximum of 1 over zone centres, u = rho (h-1)/g.
* (u_t, u_phi) solve u.u = -1 with u^t u_phi = l; u^r = u^theta = 0 is kept by
  the Boyer-Lindquist -> Kerr-Schild change, so u^{x3} = u^phi and
  u~^i = u^i - u^t g^{ti}/g^{tt} in the modified coordinates.
* Atmosphere: rho >= 1e-5 r^-3/2, u >= 1e-7 r^-5/2 (u~ = 0 outside the torus).
* u inside the torus is multiplied by 1 + 0.04 (2 xi - 1), xi uniform from
  numpy.random.default_rng(seed), drawn in C order over the interior (k, j, i).
* A_phi at (x1, x2) corners = max(rho_FM/rho_max - 0.2, 0) (unperturbed), B^1,
  B^2 from its corner curl divided by sqrt(-g), B^3 = 0, then B scaled so that
  min over zones with b^2 > 0 of 2p/b^2 equals beta_min.
"""

import math
import numpy as np

from .spec import (GridSpec, NG, NVAR, BC_OUTFLOW, BC_POLAR, BC_PERIODIC,
                   METRIC_KERR_MKS)


def horizon(a):
    return 1.0 + math.sqrt(1.0 - a * a)


def torus_grid(n1, n2, n3, a=0.9375, hslope=0.3, rout=1000.0, rin_frac=0.95):
    return GridSpec(n1, n2, n3,
                    x1min=math.log(rin_frac * horizon(a)), x1max=math.log(rout),
                    x2min=0.0, x2max=1.0, x3min=0.0, x3max=2.0 * math.pi,
                    bc=(BC_OUTFLOW, BC_OUTFLOW, BC_POLAR, BC_POLAR,
                        BC_PERIODIC, BC_PERIODIC),
                    metric=METRIC_KERR_MKS, a=a, hslope=hslope)


def mks_theta(x2, h):
    return np.pi * x2 + 0.5 * (1.0 - h) * np.sin(2.0 * np.pi * x2)


def mks_dtheta(x2, h):
    return np.pi * (1.0 + (1.0 - h) * np.cos(2.0 * np.pi * x2))


def fm_ell(a, rmax):
    """u^t u_phi of the prograde circular equatorial geodesic at rmax."""
    r = rmax
    sr = math.sqrt(r)
    den = r ** 0.75 * math.sqrt(r ** 1.5 - 3.0 * sr + 2.0 * a)
    E = (r ** 1.5 - 2.0 * sr + a) / den
    L = (r * r - 2.0 * a * sr + a * a) / den
    sig = r * r
    dl = r * r - 2.0 * r + a * a
    A = (r * r + a * a) ** 2 - a * a * dl
    gtt = -A / (sig * dl)
    gtp = -2.0 * a * r / (sig * dl)
    ut = gtt * (-E) + gtp * L
    return ut * L


def fm_lnh(r, th, a, ell, rin):
    """Fishbone-Moncrief ln h, zero at (rin, pi/2); NaN where undefined."""
    def raw(r, th):
        s2 = np.sin(th) ** 2
        c2 = np.cos(th) ** 2
        sig = r * r + a * a * c2
        dl = r * r - 2.0 * r + a * a
        A = (r * r + a * a) ** 2 - dl * a * a * s2
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.sqrt(1.0 + 4.0 * ell * ell * sig * sig * dl / (A * A * s2))
            return (0.5 * np.log((1.0 + t) / (sig * dl / A)) - 0.5 * t
                    - 2.0 * a * ell * r / A)
    return raw(r, th) - raw(np.float64(rin), np.float64(np.pi / 2))


def _bl_gcon_tphi(r, th, a):
    s2 = np.sin(th) ** 2
    sig = r * r + a * a * np.cos(th) ** 2
    dl = r * r - 2.0 * r + a * a
    A = (r * r + a * a) ** 2 - a * a * dl * s2
    gtt = -A / (sig * dl)
    gtp = -2.0 * a * r / (sig * dl)
    gpp = (dl - a * a * s2) / (sig * dl * s2)
    return gtt, gtp, gpp


def _mks_metric(x1, x2, a, h):
    """Covariant metric (4,4,...) and sqrt(-g) of Kerr in modified KS."""
    r = np.exp(x1)
    th = mks_theta(x2, h)
    dth = mks_dtheta(x2, h)
    s = np.sin(th)
    c = np.cos(th)
    s2 = s * s
    sig = r * r + a * a * c * c
    z = 2.0 * r / sig
    shape = np.broadcast(x1, x2).shape
    ks = np.zeros((4, 4) + shape)
    ks[0, 0] = -(1.0 - z)
    ks[0, 1] = ks[1, 0] = z
    ks[0, 3] = ks[3, 0] = -z * a * s2
    ks[1, 1] = 1.0 + z
    ks[1, 3] = ks[3, 1] = -a * s2 * (1.0 + z)
    ks[2, 2] = sig
    ks[3, 3] = s2 * (sig + a * a * s2 * (1.0 + z))
    lam = [np.ones(shape), r * np.ones(shape), dth * np.ones(shape), np.ones(shape)]
    g = np.empty_like(ks)
    for m in range(4):
        for n in range(4):
            g[m, n] = ks[m, n] * lam[m] * lam[n]
    gdet = sig * np.abs(s) * r * dth
    # inverse: only g^{tt} and g^{t1} are needed here
    gtt_con = -(1.0 + z)
    gt1_con = z / r
    return g, gdet, gtt_con, gt1_con


def _bsq(P, gcov, gtt_con, gt1_con):
    """b^mu b_mu for prims P (8, ...) in a metric with g^{t2} = g^{t3} = 0."""
    ut_ = P[2:5]
    qsq = np.zeros(P.shape[1:])
    for i in range(3):
        for j in range(3):
            qsq = qsq + gcov[1 + i, 1 + j] * ut_[i] * ut_[j]
    gam = np.sqrt(1.0 + qsq)
    alpha = 1.0 / np.sqrt(-gtt_con)
    ucon = np.empty((4,) + P.shape[1:])
    ucon[0] = gam / alpha
    ucon[1] = ut_[0] - gam * alpha * gt1_con
    ucon[2] = ut_[1]
    ucon[3] = ut_[2]
    ucov = np.einsum("mn...,n...->m...", gcov, ucon)
    B = P[5:8]
    bt = B[0] * ucov[1] + B[1] * ucov[2] + B[2] * ucov[3]
    bcon = np.empty_like(ucon)
    bcon[0] = bt
    for i in range(3):
        bcon[1 + i] = (B[i] + bt * ucon[1 + i]) / ucon[0]
    bcov = np.einsum("mn...,n...->m...", gcov, bcon)
    return np.einsum("m...,m...->...", bcon, bcov)


def fm_torus(n1, n2, n3, a=0.9375, hslope=0.3, rin=6.0, rmax=12.0,
             gamma=13.0 / 9.0, beta_min=100.0, seed=1, noise=0.04,
             rout=1000.0, magnetised=True):
    """Grid and padded initial prims of the torus; ghosts hold the same
    analytic data continued past the domain (used as frozen ghosts)."""
    grid = torus_grid(n1, n2, n3, a=a, hslope=hslope, rout=rout)
    x1, x2, x3 = grid.centers()
    d1, d2, _ = grid.dx
    ell = fm_ell(a, rmax)

    X2, X1 = np.meshgrid(x2, x1, indexing="ij")          # (j, i) 2-D
    r = np.exp(X1)
    th = mks_theta(X2, hslope)
    lnh = fm_lnh(r, th, a, ell, rin)
    inside = (r >= rin) & np.isfinite(lnh) & (lnh > 0.0)
    hm1 = np.where(inside, np.expm1(np.where(inside, lnh, 0.0)), 0.0)
    rho_raw = np.where(inside, (hm1 * (gamma - 1.0) / gamma) ** (1.0 / (gamma - 1.0)), 0.0)
    jin = slice(NG, NG + n2)
    iin = slice(NG, NG + n1)
    rho_max = rho_raw[jin, iin].max()

    # velocity of the constant-l torus (Boyer-Lindquist), then u~ in MKS
    gtt, gtp, gpp = _bl_gcon_tphi(r, th, a)
    with np.errstate(invalid="ignore", divide="ignore"):
        D2 = gtt * gpp - gtp * gtp
        X = (-gtt - np.sqrt(gtt * gtt - 4.0 * D2 * ell * ell)) / (2.0 * D2)
        uphi_cov = np.sqrt(X)
        ut_cov = (ell / uphi_cov - gtp * uphi_cov) / gtt
        ut_con = gtt * ut_cov + gtp * uphi_cov
        uphi_con = gtp * ut_cov + gpp * uphi_cov
    gcov, gdet, gtt_mks, gt1_mks = _mks_metric(X1, X2, a, hslope)
    ut1 = np.where(inside, -ut_con * gt1_mks / gtt_mks, 0.0)
    ut3 = np.where(inside, uphi_con, 0.0)

    shape3 = (n3 + 2 * NG, n2 + 2 * NG, n1 + 2 * NG)
    P = np.zeros((NVAR,) + shape3)
    rho2 = rho_raw / rho_max
    u2 = rho2 * hm1 / gamma
    P[0] = rho2[None]
    P[1] = u2[None]
    P[2] = ut1[None]
    P[4] = ut3[None]

    rng = np.random.default_rng(seed)
    xi = rng.random((n3, n2, n1))
    pert = np.ones(shape3)
    pert[NG:NG + n3, NG:NG + n2, NG:NG + n1] = 1.0 + noise * (2.0 * xi - 1.0)
    P[1] = np.where(inside[None], P[1] * pert, P[1])

    rfull = r[None] * np.ones(shape3)
    P[0] = np.maximum(P[0], 1e-5 * rfull ** -1.5)
    P[1] = np.maximum(P[1], 1e-7 * rfull ** -2.5)

    if magnetised:
        # A_phi at corners (x1 - dx1/2, x2 - dx2/2) of every padded zone, plus one
        c1 = grid.x1min + (np.arange(-NG, n1 + NG + 1)) * d1
        c2 = grid.x2min + (np.arange(-NG, n2 + NG + 1)) * d2
        C2, C1 = np.meshgrid(c2, c1, indexing="ij")
        rc = np.exp(C1)
        thc = mks_theta(C2, hslope)
        lnhc = fm_lnh(rc, thc, a, ell, rin)
        insc = (rc >= rin) & np.isfinite(lnhc) & (lnhc > 0.0)
        hc = np.where(insc, np.expm1(np.where(insc, lnhc, 0.0)), 0.0)
        rhoc = np.where(insc, (hc * (gamma - 1.0) / gamma) ** (1.0 / (gamma - 1.0)), 0.0) / rho_max
        A = np.maximum(rhoc - 0.2, 0.0)
        B1 = (A[1:, :-1] + A[1:, 1:] - A[:-1, :-1] - A[:-1, 1:]) / (2.0 * d2 * gdet)
        B2 = -(A[:-1, 1:] + A[1:, 1:] - A[:-1, :-1] - A[1:, :-1]) / (2.0 * d1 * gdet)
        # face fields sqrt(-g) B^d on the lower faces (the zone B above is
        # their mean over sqrt(-g)): the corner differences of A_phi
        phi1 = (A[1:, :-1] - A[:-1, :-1]) / d2
        phi2 = -(A[:-1, 1:] - A[:-1, :-1]) / d1
        P[5] = B1[None]
        P[6] = B2[None]
        gc = np.broadcast_to(gcov[:, :, None], (4, 4) + shape3)
        bsq = _bsq(P, gc, gtt_mks[None], gt1_mks[None])
        pg = (gamma - 1.0) * P[1]
        sl = (slice(NG, NG + n3), slice(NG, NG + n2), slice(NG, NG + n1))
        bi = bsq[sl]
        pi_ = pg[sl]
        m = bi > 0
        beta_min_now = np.min(2.0 * pi_[m] / bi[m])
        f = math.sqrt(beta_min_now / beta_min)
        P[5:8] *= f
        info_faces = np.zeros((3,) + shape3)
        info_faces[0] = (phi1 * f)[None]
        info_faces[1] = (phi2 * f)[None]
    else:
        info_faces = np.zeros((3,) + shape3)

    info = dict(ell=ell, rho_max_raw=rho_max, gamma=gamma, seed=seed, faces=info_faces)
    return grid, P, info
