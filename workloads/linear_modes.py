"""Linear ideal-MHD eigenmodes on a uniform flat background at rest.

The convergence tests the paper runs after every commit propagate the
Alfven, fast and slow linear modes (Readiness and Testing section).  The
eigenvector is taken from the linearised continuum equations written out
below, at rest, in flat space; it uses none of the discretisation.

Primitive perturbation X = (drho, du, du~1, du~2, du~3, dB1, dB2, dB3).  At
rest u^t = 1 + O(2), b^t = B.dv and b^i = B^i + O(2), so with
w = rho + u + p and p = (gamma - 1) u the linearised conserved variables and
fluxes of the ideal GRMHD system (stress-energy tensor of the EGRMHD
section, ideal part) are

    dU_rho = drho                          dF^d_rho = rho dv^d
    dU_E   = -(du + B.dB)                  dF^d_E   = -[(w + B^2) dv^d - (B.dv) B^d] + rho dv^d
    dU_i   = (w + B^2) dv^i - (B.dv) B^i    dF^d_i   = (dp + B.dB) delta_di - B^d dB^i - dB^d B^i
    dU_Bk  = dB^k                          dF^d_Bk  = B^k dv^d - B^d dv^k

and a plane wave exp(i(k.x - omega t)) solves (sum_d k_d A_d) X = omega A_0 X.
"""

import math

import numpy as np

from .spec import GridSpec, NG, NVAR, BC_PERIODIC, METRIC_MINKOWSKI

MODES = ("entropy", "slow", "alfven", "fast")


def _jacobians(rho, u, B, gamma):
    """A_0 = dU/dP and A_d = dF^d/dP at rest (flat space), by hand."""
    p = (gamma - 1.0) * u
    w = rho + u + p
    B = np.asarray(B, float)
    b2 = B @ B
    A0 = np.zeros((NVAR, NVAR))
    A0[0, 0] = 1.0
    A0[1, 1] = -1.0
    A0[1, 5:8] = -B
    for i in range(3):
        A0[2 + i, 2 + i] += w + b2
        A0[2 + i, 2:5] -= B[i] * B
        A0[5 + i, 5 + i] = 1.0
    Ad = []
    for d in range(3):
        A = np.zeros((NVAR, NVAR))
        A[0, 2 + d] = rho
        # energy flux: -[(w + b2) dv^d - (B.dv) B^d] + rho dv^d
        A[1, 2 + d] += -(w + b2) + rho
        A[1, 2:5] += B[d] * B
        for i in range(3):
            # momentum flux (dp + B.dB) delta_di - B^d dB^i - dB^d B^i
            if i == d:
                A[2 + i, 1] += gamma - 1.0
                A[2 + i, 5:8] += B
            A[2 + i, 5 + i] -= B[d]
            A[2 + i, 5 + d] -= B[i]
            # induction flux B^k dv^d - B^d dv^k
            A[5 + i, 2 + d] += B[i]
            A[5 + i, 2 + i] -= B[d]
        Ad.append(A)
    return A0, Ad


def mode_eigensystem(rho=1.0, u=1.0, B=(1.0, 0.0, 0.0), gamma=4.0 / 3.0,
                     k=(2 * np.pi, 2 * np.pi, 0.0)):
    """Phase speeds omega/|k| and real eigenvectors of the linear system."""
    A0, Ad = _jacobians(rho, u, B, gamma)
    K = sum(kd * A for kd, A in zip(k, Ad))
    M = np.linalg.solve(A0, K)
    lam, vec = np.linalg.eig(M)
    kn = np.linalg.norm(k)
    order = np.argsort(lam.real)
    lam = lam.real[order] / kn
    vec = vec[:, order]
    out = []
    for j in range(NVAR):
        v = vec[:, j]
        v = v / v[np.argmax(np.abs(v))]      # remove the arbitrary complex phase
        out.append(v.real)
    return lam, np.array(out)


def _normalise(r):
    r = np.asarray(r, float)
    r = r / np.linalg.norm(r)
    for idx in (0, 1, 4, 7):               # sign rule: first nonzero of these > 0
        if abs(r[idx]) > 1e-12:
            if r[idx] < 0:
                r = -r
            break
    r[np.abs(r) < 1e-15] = 0.0
    return r


def select_mode(name, rho=1.0, u=1.0, B=(1.0, 0.0, 0.0), gamma=4.0 / 3.0,
                k=(2 * np.pi, 2 * np.pi, 0.0)):
    """(phase speed, unit eigenvector) of a named right-going mode."""
    if name == "entropy":
        r = np.zeros(NVAR)
        r[0] = 1.0
        return 0.0, r
    lam, vec = mode_eigensystem(rho, u, B, gamma, k)
    pos = [(l, v) for l, v in zip(lam, vec) if l > 1e-8]
    pos.sort(key=lambda t: t[0])
    if len(pos) != 3:
        raise ValueError("unexpected eigenstructure: %r" % (lam,))
    which = {"slow": 0, "alfven": 1, "fast": 2}[name]
    l, v = pos[which]
    return float(l), _normalise(v)


def linear_mode(name, n, ndim=3, amp=1e-4, rho=1.0, u=1.0, B=(1.0, 0.0, 0.0),
                gamma=4.0 / 3.0, kvec=(2 * np.pi, 2 * np.pi, 0.0)):
    """Grid, initial padded prims and exact solution for a linear mode.

    Unit periodic box [0,1)^ndim (n zones per active axis, one zone on the
    others), background prims (rho, u, 0, 0, 0, B), perturbation
    amp * r * cos(k.x) at zone centres.  Returns (grid, prims, exact) where
    exact(t) gives the padded exact prims at time t.
    """
    n1 = n
    n2 = n if ndim >= 2 else 1
    n3 = n if ndim >= 3 else 1
    g = GridSpec(n1, n2, n3, bc=(BC_PERIODIC,) * 6, metric=METRIC_MINKOWSKI)
    speed, r = select_mode(name, rho, u, B, gamma, kvec)
    omega = speed * np.linalg.norm(kvec)
    x1, x2, x3 = g.centers()
    X3, X2, X1 = np.meshgrid(x3, x2, x1, indexing="ij")
    P0 = np.array([rho, u, 0.0, 0.0, 0.0, B[0], B[1], B[2]])

    def exact(t):
        phase = kvec[0] * X1 + kvec[1] * X2 + kvec[2] * X3 - omega * t
        c = np.cos(phase)
        return P0[:, None, None, None] + amp * r[:, None, None, None] * c[None]

    return g, exact(0.0), exact, dict(speed=speed, omega=omega, r=r)


def linear_mode_faces(name, n, ndim=3, amp=1e-4, rho=1.0, u=1.0, B=(1.0, 0.0, 0.0),
                      gamma=4.0 / 3.0, kvec=(2 * np.pi, 2 * np.pi, 0.0)):
    """linear_mode plus the face fields of face-centred constrained transport:
    faces[d] = the average of B^d over the lower d-face of every padded zone
    (flat space, so sqrt(-g) = 1), i.e. B0_d + amp r_Bd cos(k.x_face) times
    sinc(k_e dx_e / 2) for the two other axes e.  Face averages of a
    divergence-free field have zero discrete face divergence.  Returns
    (grid, prims, faces, exact, info)."""
    g, P, exact, info = linear_mode(name, n, ndim=ndim, amp=amp, rho=rho, u=u, B=B, gamma=gamma,
                                    kvec=kvec)
    r = info["r"]
    x1, x2, x3 = g.centers()
    dx = g.dx
    centres = [x1, x2, x3]
    faces = np.zeros((3,) + P.shape[1:])
    for d in range(3):
        xs = [c.copy() for c in centres]
        xs[d] = xs[d] - 0.5 * dx[d]
        X3, X2, X1 = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
        fac = 1.0
        for e in range(3):
            if e != d:
                h = 0.5 * kvec[e] * dx[e]
                fac *= math.sin(h) / h if h != 0.0 else 1.0
        phase = kvec[0] * X1 + kvec[1] * X2 + kvec[2] * X3
        faces[d] = B[d] + amp * r[5 + d] * fac * np.cos(phase)
    return g, P, faces, exact, info
