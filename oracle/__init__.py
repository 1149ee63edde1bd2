"""TEST INFRASTRUCTURE ONLY: ctypes front end of the FP64 CPU oracle.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  `build()` compiles harm_oracle.cpp with g++ (OpenMP, no
fast-math, no FMA) into liboracle.so next to it.  Two more builds of the
same source serve as measuring instruments: the counting build (every
floating-point operation tallied) and the FMA build (g++ free to contract
a*b + c into fused multiply-adds), whose distance from the plain build is
the rounding noise floor of a result.
"""

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "harm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_COUNT = os.path.join(HERE, "liboracle_count.so")
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")


def build(counting=False, fma=False):
    out = LIB_COUNT if counting else (LIB_FMA if fma else LIB)
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=fast" if fma else "-ffp-contract=off", "-o", out, SRC]
    if fma:
        cmd[1:1] = ["-mfma"]
    if counting:
        cmd[1:1] = ["-DORACLE_COUNTING"]
    else:
        cmd[1:1] = ["-fopenmp"]
    subprocess.check_call(cmd, cwd=HERE)
    return out


class Cfg(C.Structure):
    _fields_ = [("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int),
                ("x1min", C.c_double), ("x1max", C.c_double),
                ("x2min", C.c_double), ("x2max", C.c_double),
                ("x3min", C.c_double), ("x3max", C.c_double),
                ("bc", C.c_int * 6), ("metric", C.c_int),
                ("a", C.c_double), ("hslope", C.c_double),
                ("gam", C.c_double), ("recon", C.c_int),
                ("weno_eps", C.c_double), ("newton_tol", C.c_double),
                ("newton_maxit", C.c_int), ("cfl", C.c_double),
                ("nthreads", C.c_int), ("inverter", C.c_int),
                ("kastaun_wmax", C.c_double), ("floors", C.c_int),
                ("rho_min_geom", C.c_double), ("u_min_geom", C.c_double),
                ("bsq_over_rho_max", C.c_double), ("bsq_over_u_max", C.c_double),
                ("u_over_rho_max", C.c_double), ("gamma_max", C.c_double),
                ("fofc", C.c_int), ("ct", C.c_int), ("integrator", C.c_int),
                ("tau_r", C.c_double), ("chi_emhd", C.c_double), ("nu_emhd", C.c_double)]

INV_1DW, INV_KASTAUN, INV_IMPLICIT = 0, 1, 2
RECON_DONOR = 2
RECON_WENOZ = 3
RECON_VL = 4
RECON_MP5 = 5
RECON_PPM = 6
RECON_PPMX = 7
CT_FLUX, CT_FACE_AVG, CT_FACE_GS = 0, 1, 2
INTEG_SSPRK2, INTEG_PC, INTEG_RK1, INTEG_SSPRK54 = 0, 1, 2, 3
FL_RHO, FL_U, FL_FLUID_FRAME, FL_GAMMA, FL_TEMP = 1, 2, 4, 8, 16
# floor and ceiling defaults (HARM-family values; the paper states none)
FLOOR_DEFAULTS = dict(rho_min_geom=1e-6, u_min_geom=1e-8, bsq_over_rho_max=100.0,
                      bsq_over_u_max=5000.0, u_over_rho_max=100.0, gamma_max=50.0)


_lib = None
_lib_count = None
_lib_fma = None

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def _declare(lib):
    P = C.POINTER(Cfg)
    lib.orc_run.argtypes = [P, _D, C.c_double, C.c_int, _D, _I]
    lib.orc_run.restype = C.c_long
    lib.orc_estimate_dt.argtypes = [P, _D]
    lib.orc_estimate_dt.restype = C.c_double
    lib.orc_fill_ghosts.argtypes = [P, _D]
    lib.orc_divb.argtypes = [P, _D, _D, _D, _D]
    lib.orc_fluxes.argtypes = [P, _D, _D, C.c_int]
    lib.orc_prims_to_cons.argtypes = [P, _D, _D]
    lib.orc_cons_to_prims.argtypes = [P, _D, _D, _D, _I]
    lib.orc_cons_to_prims.restype = C.c_long
    lib.orc_geom.argtypes = [P, C.c_double, C.c_double, _D, _D, _D, _D]
    lib.orc_conn.argtypes = [P, C.c_double, C.c_double, _D]
    lib.orc_point_flux.argtypes = [P, _D, C.c_double, C.c_double, C.c_int, _D, _D, _D]
    lib.orc_point_source.argtypes = [P, _D, C.c_double, C.c_double, _D]
    lib.orc_point_u_to_p.argtypes = [P, _D, _D, C.c_double, C.c_double, _D]
    lib.orc_point_u_to_p.restype = C.c_int
    lib.orc_point_floors.argtypes = [P, _D, C.c_double, C.c_double]
    lib.orc_point_floors.restype = C.c_int
    lib.orc_last_stats.argtypes = [C.POINTER(C.c_longlong)]
    lib.orc_run_emhd.argtypes = [P, _D, _D, C.c_double, C.c_int, _D]
    lib.orc_run_emhd.restype = C.c_long
    lib.orc_cons_emhd.argtypes = [P, _D, _D, _D]
    lib.orc_emhd_targets.argtypes = [P, _D, C.c_int, C.c_int, C.c_int, _D]
    lib.orc_run_face.argtypes = [P, _D, _D, C.c_double, C.c_int, _D, _I]
    lib.orc_run_face.restype = C.c_long
    lib.orc_face_divb.argtypes = [P, _D, _D, _D]
    lib.orc_edge_emfs.argtypes = [P, _D, _D, _D]
    lib.orc_qr_solve.argtypes = [_D, _D, _D]
    lib.orc_qr_solve.restype = C.c_int
    lib.orc_weno5.argtypes = [C.c_double] * 6
    lib.orc_weno5.restype = C.c_double
    lib.orc_mc_slope.argtypes = [C.c_double] * 3
    lib.orc_mc_slope.restype = C.c_double
    lib.orc_ssprk54_coefficients.argtypes = [_D]
    lib.orc_ssprk54_coefficients.restype = None
    lib.orc_wenoz.argtypes = [C.c_double] * 6
    lib.orc_wenoz.restype = C.c_double
    lib.orc_vl_slope.argtypes = [C.c_double] * 3
    lib.orc_vl_slope.restype = C.c_double
    lib.orc_mp5.argtypes = [C.c_double] * 5
    lib.orc_mp5.restype = C.c_double
    lib.orc_ppm_edges.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)] * 2
    lib.orc_ppm_edges.restype = None
    lib.orc_ppmx_edges.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)] * 2
    lib.orc_ppmx_edges.restype = None
    L = C.POINTER(C.c_longlong)
    lib.orc_count_face.argtypes = [P, _D, C.c_int, C.c_int, C.c_int, C.c_int, L]
    lib.orc_count_zone_update.argtypes = [P, _D, C.c_int, C.c_int, C.c_int, C.c_double, L]
    return lib


def lib(counting=False, fma=False):
    global _lib, _lib_count, _lib_fma
    if fma:
        if _lib_fma is None:
            if not os.path.exists(LIB_FMA) or os.path.getmtime(LIB_FMA) < os.path.getmtime(SRC):
                build(fma=True)
            _lib_fma = _declare(C.CDLL(LIB_FMA))
        return _lib_fma
    if counting:
        if _lib_count is None:
            if not os.path.exists(LIB_COUNT) or os.path.getmtime(LIB_COUNT) < os.path.getmtime(SRC):
                build(counting=True)
            _lib_count = _declare(C.CDLL(LIB_COUNT))
        return _lib_count
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _declare(C.CDLL(LIB))
    return _lib


def cfg(grid, gam=4.0 / 3.0, recon=0, weno_eps=1e-26, newton_tol=1e-14,
        newton_maxit=30, cfl=0.9, nthreads=None, inverter=INV_1DW, kastaun_wmax=1e3,
        floors=False, fofc=False, ct=CT_FLUX, integrator=INTEG_SSPRK2, tau_r=1.0, chi_emhd=0.0,
        nu_emhd=0.0, **floor_params):
    c = Cfg()
    c.n1, c.n2, c.n3 = grid.n1, grid.n2, grid.n3
    c.x1min, c.x1max = grid.x1min, grid.x1max
    c.x2min, c.x2max = grid.x2min, grid.x2max
    c.x3min, c.x3max = grid.x3min, grid.x3max
    for i in range(6):
        c.bc[i] = int(grid.bc[i])
    c.metric = int(grid.metric)
    c.a, c.hslope = grid.a, grid.hslope
    c.gam, c.recon, c.weno_eps = gam, int(recon), weno_eps
    c.newton_tol, c.newton_maxit, c.cfl = newton_tol, newton_maxit, cfl
    c.nthreads = nthreads or os.cpu_count() or 1
    c.inverter, c.kastaun_wmax = int(inverter), float(kastaun_wmax)
    c.floors, c.fofc = int(bool(floors)), int(bool(fofc))
    c.ct = int(ct)
    c.integrator = int(integrator)
    if c.integrator == INTEG_SSPRK54 and (c.floors or c.fofc or c.ct != CT_FLUX):
        raise ValueError("SSPRK(5,4) takes the plain Flux-CT step only")
    c.tau_r, c.chi_emhd, c.nu_emhd = float(tau_r), float(chi_emhd), float(nu_emhd)
    fp = dict(FLOOR_DEFAULTS)
    for k, v in floor_params.items():
        if k not in fp:
            raise TypeError(f"unknown floor parameter {k}")
        fp[k] = v
    for k, v in fp.items():
        setattr(c, k, float(v))
    return c


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def run(c, prims, dt, nsteps=1, counting=False, flags=False, fma=False):
    """Advance a copy of prims; returns (prims, fails, dts[, per-zone flags]).
    fma: with the FMA build (the rounding noise floor)."""
    P = np.ascontiguousarray(prims, dtype=np.float64).copy()
    dts = np.zeros(max(nsteps, 1))
    fl = np.zeros(P.shape[1:], dtype=np.int32) if flags else None
    fails = lib(counting, fma).orc_run(C.byref(c), _ptr(P), float(dt), int(nsteps), _ptr(dts),
                                       fl.ctypes.data_as(_I) if flags else None)
    if flags:
        return P, int(fails), dts, fl
    return P, int(fails), dts


def run_emhd(c, prims, extra, dt, nsteps=1, fma=False):
    """Extended GRMHD (predictor-corrector): advance copies of prims and of
    the extra variables ([2][padded]: rescaled heat flux and pressure
    anisotropy) with the closure constants c.tau_r, c.chi_emhd, c.nu_emhd;
    returns (prims, extra, fails, dts)."""
    P = np.ascontiguousarray(prims, dtype=np.float64).copy()
    X = np.ascontiguousarray(extra, dtype=np.float64).copy()
    assert X.shape == (2,) + P.shape[1:]
    dts = np.zeros(max(nsteps, 1))
    fails = lib(fma=fma).orc_run_emhd(C.byref(c), _ptr(P), _ptr(X), float(dt), int(nsteps), _ptr(dts))
    return P, X, int(fails), dts


def emhd_targets(c, prims, i, j, k):
    """Extended GRMHD targets at interior zone (i, j, k): the rescaled
    heat-flux and anisotropy targets and the spatial part of div u."""
    P = np.ascontiguousarray(prims, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_emhd_targets(C.byref(c), _ptr(P), int(i), int(j), int(k), _ptr(out))
    return out[0], out[1], out[2]


def cons_emhd(c, prims, extra):
    """Conserved variables [10][padded] of Extended GRMHD at interior zones."""
    P = np.ascontiguousarray(prims, dtype=np.float64)
    X = np.ascontiguousarray(extra, dtype=np.float64)
    out = np.zeros((10,) + P.shape[1:])
    lib().orc_cons_emhd(C.byref(c), _ptr(P), _ptr(X), _ptr(out))
    return out


def run_face(c, prims, faces, dt, nsteps=1, flags=False, fma=False):
    """Face-centred CT: advance copies of prims and face fields
    ([3][padded], sqrt(-g) B^d on lower d-faces); returns (prims, faces,
    fails, dts[, flags])."""
    P = np.ascontiguousarray(prims, dtype=np.float64).copy()
    Fc = np.ascontiguousarray(faces, dtype=np.float64).copy()
    assert Fc.shape == (3,) + P.shape[1:]
    dts = np.zeros(max(nsteps, 1))
    fl = np.zeros(P.shape[1:], dtype=np.int32) if flags else None
    fails = lib(fma=fma).orc_run_face(C.byref(c), _ptr(P), _ptr(Fc), float(dt), int(nsteps), _ptr(dts),
                               fl.ctypes.data_as(_I) if flags else None)
    if flags:
        return P, Fc, int(fails), dts, fl
    return P, Fc, int(fails), dts


def edge_emfs(c, prims, faces):
    """Edge EMFs [3][padded] (E1, E2, E3) of the face-centred scheme c.ct."""
    P = np.ascontiguousarray(prims, dtype=np.float64)
    F = np.ascontiguousarray(faces, dtype=np.float64)
    out = np.zeros(F.shape)
    lib().orc_edge_emfs(C.byref(c), _ptr(P), _ptr(F), _ptr(out))
    return out


def face_divb(c, faces):
    F = np.ascontiguousarray(faces, dtype=np.float64)
    mx, mean = C.c_double(), C.c_double()
    lib().orc_face_divb(C.byref(c), _ptr(F), C.byref(mx), C.byref(mean))
    return mx.value, mean.value


def last_stats(counting=False):
    """Counters of the last run: failed inversions, zones the floors acted
    on, zones the first-order flux correction marked, fluid-frame fallbacks
    of the floors."""
    out = (C.c_longlong * 4)()
    lib(counting).orc_last_stats(out)
    return dict(fails=out[0], floor_hits=out[1], fofc_zones=out[2], fluid_frame=out[3])


def estimate_dt(c, prims):
    P = np.ascontiguousarray(prims, dtype=np.float64).copy()
    return lib().orc_estimate_dt(C.byref(c), _ptr(P))


def fill_ghosts(c, prims):
    P = np.ascontiguousarray(prims, dtype=np.float64).copy()
    lib().orc_fill_ghosts(C.byref(c), _ptr(P))
    return P


def divb(c, prims, field=False):
    P = np.ascontiguousarray(prims, dtype=np.float64)
    mx, mean = C.c_double(), C.c_double()
    f = np.zeros(P.shape[1:]) if field else None
    lib().orc_divb(C.byref(c), _ptr(P), C.byref(mx), C.byref(mean),
                   _ptr(f) if field else None)
    return (mx.value, mean.value, f) if field else (mx.value, mean.value)


def fluxes(c, prims, ct=True):
    P = np.ascontiguousarray(prims, dtype=np.float64)
    F = np.zeros((3,) + P.shape)
    lib().orc_fluxes(C.byref(c), _ptr(P), _ptr(F), int(ct))
    return F


def prims_to_cons(c, prims):
    P = np.ascontiguousarray(prims, dtype=np.float64)
    U = np.zeros_like(P)
    lib().orc_prims_to_cons(C.byref(c), _ptr(P), _ptr(U))
    return U


def cons_to_prims(c, cons, guess):
    U = np.ascontiguousarray(cons, dtype=np.float64)
    G = np.ascontiguousarray(guess, dtype=np.float64)
    P = np.zeros_like(U)
    flags = np.zeros(U.shape[1:], dtype=np.int32)
    n = lib().orc_cons_to_prims(C.byref(c), _ptr(U), _ptr(G), _ptr(P),
                                flags.ctypes.data_as(_I))
    return P, int(n), flags


def geom(c, x1, x2):
    gcov = np.zeros(16)
    gcon = np.zeros(16)
    gdet, alpha = C.c_double(), C.c_double()
    lib().orc_geom(C.byref(c), x1, x2, _ptr(gcov), _ptr(gcon), C.byref(gdet), C.byref(alpha))
    return gcov.reshape(4, 4), gcon.reshape(4, 4), gdet.value, alpha.value


def conn(c, x1, x2):
    out = np.zeros(64)
    lib().orc_conn(C.byref(c), x1, x2, _ptr(out))
    return out.reshape(4, 4, 4)


def point_flux(c, prims, x1, x2, d):
    p = np.ascontiguousarray(prims, dtype=np.float64)
    out = np.zeros(8)
    cp, cm = C.c_double(), C.c_double()
    lib().orc_point_flux(C.byref(c), _ptr(p), x1, x2, int(d), _ptr(out), C.byref(cp), C.byref(cm))
    return out, cp.value, cm.value


def point_source(c, prims, x1, x2):
    p = np.ascontiguousarray(prims, dtype=np.float64)
    out = np.zeros(8)
    lib().orc_point_source(C.byref(c), _ptr(p), x1, x2, _ptr(out))
    return out


def point_u_to_p(c, cons, guess, x1, x2):
    u = np.ascontiguousarray(cons, dtype=np.float64)
    g = np.ascontiguousarray(guess, dtype=np.float64)
    out = np.zeros(8)
    r = lib().orc_point_u_to_p(C.byref(c), _ptr(u), _ptr(g), x1, x2, _ptr(out))
    return out, r


def point_floors(c, prims, x1, x2):
    """Floors and ceilings of one zone's prims: (new prims, mask)."""
    p = np.array(prims, dtype=np.float64)
    m = lib().orc_point_floors(C.byref(c), _ptr(p), x1, x2)
    return p, m


def qr_solve(A, b):
    """The implicit solver's pivoted-QR solve of a 5 x 5 system: (y, ok)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    y = np.zeros(5)
    ok = lib().orc_qr_solve(_ptr(A), _ptr(b), _ptr(y))
    return y, bool(ok)


def weno5(a, b, c_, d, e, eps=1e-26):
    return lib().orc_weno5(a, b, c_, d, e, eps)


def ssprk54_coefficients():
    """The SSPRK(5,4) step's Shu-Osher coefficients, as the step uses them:
    c1, (a_k, b_k, c_k) for k = 2, 3, 4, then d2, d3, e3, d4, e4."""
    out = np.zeros(15)
    lib().orc_ssprk54_coefficients(_ptr(out))
    return out


def mc_slope(l, c_, r):
    return lib().orc_mc_slope(l, c_, r)


def wenoz(a, b, c_, d, e, eps=1e-26):
    return lib().orc_wenoz(a, b, c_, d, e, eps)


def vl_slope(l, c_, r):
    return lib().orc_vl_slope(l, c_, r)


def mp5(a, b, c_, d, e):
    return lib().orc_mp5(a, b, c_, d, e)


def ppm_edges(a, b, c_, d, e):
    """(left, right) edge values of the middle zone."""
    l, r = C.c_double(), C.c_double()
    lib().orc_ppm_edges(a, b, c_, d, e, C.byref(l), C.byref(r))
    return l.value, r.value


def ppmx_edges(a, b, c_, d, e):
    """PPMX (Colella & Sekora 2008): (left, right) edge values of the
    middle zone."""
    l, r = C.c_double(), C.c_double()
    lib().orc_ppmx_edges(a, b, c_, d, e, C.byref(l), C.byref(r))
    return l.value, r.value


def count_face(c, prims, d, i, j, k):
    """(add, mul, div, sqrt, transcendental) of one face flux (counting build)."""
    out = (C.c_longlong * 5)()
    P = np.ascontiguousarray(prims, dtype=np.float64)
    lib(True).orc_count_face(C.byref(c), _ptr(P), d, i, j, k, out)
    return list(out)


def count_zone_update(c, prims, i, j, k, dt):
    out = (C.c_longlong * 5)()
    P = np.ascontiguousarray(prims, dtype=np.float64)
    lib(True).orc_count_zone_update(C.byref(c), _ptr(P), i, j, k, float(dt), out)
    return list(out)
