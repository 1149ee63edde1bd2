"""ctypes binding of libgrmhd.so (include/grmhd.h): argument marshalling only.

Every computation runs in the HIP library; this module passes raw device
pointers of torch tensors and the current torch stream.  There is no
fallback: importing it without the built library raises.
"""

import atexit
import ctypes as C
import os
import sys
import weakref

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrmhd.so")

OK, E_ARG, E_HIP, E_STATE, E_NOMEM = 0, -1, -2, -3, -4
METRIC_MINKOWSKI, METRIC_KERR_MKS = 0, 1
RECON_MC, RECON_WENO5, RECON_DONOR, RECON_WENOZ, RECON_VL, RECON_MP5, RECON_PPM, RECON_PPMX = range(8)
PREC_FP64, PREC_MIXED = 0, 1
INV_1DW, INV_KASTAUN, INV_IMPLICIT = 0, 1, 2
CT_FLUX, CT_FACE_AVG, CT_FACE_GS = 0, 1, 2
INTEG_SSPRK2, INTEG_PC, INTEG_RK1, INTEG_SSPRK54 = 0, 1, 2, 3
BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_FROZEN = 0, 1, 2, 3
NG, NVAR = 3, 8


class GrmhdError(RuntimeError):
    pass


class grmhd_grid(C.Structure):
    _fields_ = [("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int), ("ng", C.c_int),
                ("x1min", C.c_double), ("x1max", C.c_double), ("x2min", C.c_double),
                ("x2max", C.c_double), ("x3min", C.c_double), ("x3max", C.c_double),
                ("bc", C.c_int * 6)]


class grmhd_metric(C.Structure):
    _fields_ = [("metric", C.c_int), ("a", C.c_double), ("hslope", C.c_double)]


class grmhd_params(C.Structure):
    _fields_ = [("gamma_ad", C.c_double), ("cfl", C.c_double), ("weno_eps", C.c_double),
                ("newton_tol", C.c_double), ("newton_maxit", C.c_int), ("recon", C.c_int),
                ("precision", C.c_int), ("floors", C.c_int), ("inverter", C.c_int),
                ("kastaun_wmax", C.c_double), ("rho_min_geom", C.c_double),
                ("u_min_geom", C.c_double), ("bsq_over_rho_max", C.c_double),
                ("bsq_over_u_max", C.c_double), ("u_over_rho_max", C.c_double),
                ("gamma_max", C.c_double), ("fofc", C.c_int), ("ct", C.c_int),
                ("integrator", C.c_int), ("egrmhd", C.c_int), ("tau_r", C.c_double),
                ("chi_emhd", C.c_double), ("nu_emhd", C.c_double)]


# floor and ceiling defaults (HARM-family values; the paper states none)
FLOOR_DEFAULTS = dict(rho_min_geom=1e-6, u_min_geom=1e-8, bsq_over_rho_max=100.0,
                      bsq_over_u_max=5000.0, u_over_rho_max=100.0, gamma_max=50.0)


def make_params(gamma_ad, cfl, weno_eps, newton_tol, newton_maxit, recon, precision, inverter,
                kastaun_wmax, floors=False, fofc=False, ct=CT_FLUX, integrator=INTEG_SSPRK2,
                egrmhd=False, tau_r=1.0, chi_emhd=0.0, nu_emhd=0.0, **floor_params):
    fp = dict(FLOOR_DEFAULTS)
    for k, v in floor_params.items():
        if k not in fp:
            raise TypeError(f"unknown floor parameter {k}")
        fp[k] = v
    return grmhd_params(float(gamma_ad), float(cfl), float(weno_eps), float(newton_tol),
                        int(newton_maxit), int(recon), int(precision), int(bool(floors)),
                        int(inverter), float(kastaun_wmax), *(float(fp[k]) for k in FLOOR_DEFAULTS),
                        int(bool(fofc)), int(ct), int(integrator), int(bool(egrmhd)),
                        float(tau_r), float(chi_emhd), float(nu_emhd))


EXPORTS = ("grmhd_workspace_bytes", "grmhd_create", "grmhd_load_prims", "grmhd_step",
           "grmhd_estimate_dt", "grmhd_step_cfl", "grmhd_last_dt", "grmhd_get_prims", "grmhd_divb", "grmhd_get_status",
           "grmhd_get_counters", "grmhd_load_faces", "grmhd_get_faces", "grmhd_face_divb",
           "grmhd_load_extended", "grmhd_get_extended",
           "grmhd_reset_status", "grmhd_prims_to_cons", "grmhd_cons_to_prims", "grmhd_fluxes",
           "grmhd_pack_workspace_bytes", "grmhd_pack_create", "grmhd_pack_set_tiles",
           "grmhd_pack_load_prims", "grmhd_pack_step", "grmhd_pack_get_prims",
           "grmhd_pack_get_status", "grmhd_pack_info", "grmhd_pack_destroy",
           "grmhd_pack_exchange_bytes", "grmhd_pack_set_exchange",
           "grmhd_vjp_workspace_bytes", "grmhd_step_vjp", "grmhd_set_schedule", "grmhd_cfl_dt_noalloc", "grmhd_timing", "grmhd_timing_report", "grmhd_strerror", "grmhd_destroy")


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2408_01361_amd.build.build()")
    lib = C.CDLL(path)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong)
    G, M, P = C.POINTER(grmhd_grid), C.POINTER(grmhd_metric), C.POINTER(grmhd_params)
    sig = {
        "grmhd_workspace_bytes": (C.c_size_t, [G, P]),
        "grmhd_create": (C.c_int, [C.POINTER(vp), G, M, P, vp, C.c_size_t, vp]),
        "grmhd_load_prims": (C.c_int, [vp, vp]),
        "grmhd_step": (C.c_int, [vp, C.c_double]),
        "grmhd_estimate_dt": (C.c_int, [vp, dp]),
        "grmhd_step_cfl": (C.c_int, [vp]),
        "grmhd_last_dt": (C.c_int, [vp, dp]),
        "grmhd_get_prims": (C.c_int, [vp, vp]),
        "grmhd_divb": (C.c_int, [vp, vp, dp, dp]),
        "grmhd_get_status": (C.c_int, [vp, ip, ip]),
        "grmhd_get_counters": (C.c_int, [vp, ip]),
        "grmhd_load_extended": (C.c_int, [vp, vp]),
        "grmhd_get_extended": (C.c_int, [vp, vp]),
        "grmhd_load_faces": (C.c_int, [vp, vp]),
        "grmhd_get_faces": (C.c_int, [vp, vp]),
        "grmhd_face_divb": (C.c_int, [vp, dp, dp]),
        "grmhd_reset_status": (C.c_int, [vp]),
        "grmhd_prims_to_cons": (C.c_int, [vp, vp, vp]),
        "grmhd_cons_to_prims": (C.c_int, [vp, vp, vp, vp, vp, ip]),
        "grmhd_fluxes": (C.c_int, [vp, vp, vp]),
        "grmhd_pack_workspace_bytes": (C.c_size_t, [C.c_int, C.POINTER(C.c_int)]),
        "grmhd_pack_create": (C.c_int, [C.POINTER(vp), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        G, M, P, vp, C.c_size_t, vp]),
        "grmhd_pack_set_tiles": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int]),
        "grmhd_pack_load_prims": (C.c_int, [vp, vp]),
        "grmhd_pack_step": (C.c_int, [vp, C.c_double]),
        "grmhd_pack_get_prims": (C.c_int, [vp, vp]),
        "grmhd_pack_get_status": (C.c_int, [vp, ip]),
        "grmhd_pack_info": (C.c_int, [vp, C.POINTER(C.c_int), ip]),
        "grmhd_pack_destroy": (C.c_int, [vp]),
        "grmhd_pack_exchange_bytes": (C.c_size_t, [G]),
        "grmhd_pack_set_exchange": (C.c_int, [vp, vp, C.c_size_t]),
        "grmhd_vjp_workspace_bytes": (C.c_size_t, [G, P]),
        "grmhd_step_vjp": (C.c_int, [vp, vp, C.c_double, vp, vp, dp, vp, C.c_size_t]),
        "grmhd_set_schedule": (C.c_int, [vp, C.c_int, C.c_int]),
        "grmhd_cfl_dt_noalloc": (C.c_int, [G, M, P, vp, dp, vp]),
        "grmhd_timing": (C.c_int, [vp, C.c_int]),
        "grmhd_timing_report": (C.c_int, [vp, dp, ip, C.c_int]),
        "grmhd_strerror": (C.c_char_p, [C.c_int]),
        "grmhd_destroy": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


# Contexts and packs still open.  They are closed by an exit handler, which
# runs while the HIP runtime is still up; a finalizer that runs later, during
# interpreter shutdown, makes no HIP call (the process is ending anyway).
_open = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_open):
        obj.close()


def _check(rc):
    if rc != OK:
        raise GrmhdError(f"grmhd error {rc}: {lib().grmhd_strerror(rc).decode()}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise GrmhdError("device tensor expected")
    if not t.is_contiguous():
        raise GrmhdError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def make_grid(spec):
    """grmhd_grid from any object with n1..n3, x?min/x?max and bc."""
    g = grmhd_grid()
    g.n1, g.n2, g.n3, g.ng = spec.n1, spec.n2, spec.n3, NG
    g.x1min, g.x1max, g.x2min, g.x2max = spec.x1min, spec.x1max, spec.x2min, spec.x2max
    g.x3min, g.x3max = spec.x3min, spec.x3max
    for i in range(6):
        g.bc[i] = int(spec.bc[i])
    return g


def cfl_dt_noalloc(spec, gamma_ad, prims, recon=RECON_WENO5, cfl=0.9, stream=None, **kw):
    """CFL step of a device prims tensor without a context or any allocation
    (grmhd_cfl_dt_noalloc); keyword options as for Grmhd."""
    grid = make_grid(spec)
    metric = grmhd_metric(int(spec.metric), float(spec.a), float(spec.hslope))
    params = make_params(gamma_ad, cfl, kw.pop("weno_eps", 1e-26), kw.pop("newton_tol", 1e-14),
                         kw.pop("newton_maxit", 30), recon, kw.pop("precision", PREC_FP64),
                         kw.pop("inverter", INV_1DW), kw.pop("kastaun_wmax", 1e3), **kw)
    if prims.dtype != torch.float64:
        raise GrmhdError("float64 prims expected")
    st = stream if stream is not None else torch.cuda.current_stream(prims.device)
    out = C.c_double()
    _check(lib().grmhd_cfl_dt_noalloc(C.byref(grid), C.byref(metric), C.byref(params), _ptr(prims),
                                      C.byref(out), C.c_void_p(st.cuda_stream)))
    return out.value


class Grmhd:
    """One grid's state and workspace on a CUDA (HIP) device.

    Python owns the workspace tensor; the library borrows it for the
    context's lifetime and enqueues on the torch stream current at creation.

    Options (the fields of grmhd_params in include/grmhd.h): recon
    (RECON_MC, RECON_WENO5, RECON_DONOR, RECON_WENOZ, RECON_VL, RECON_MP5,
    RECON_PPM, RECON_PPMX), precision
    (PREC_FP64, PREC_MIXED),
    inverter (INV_1DW, INV_KASTAUN, INV_IMPLICIT), floors (with the keyword
    floor parameters of FLOOR_DEFAULTS), fofc (first-order flux correction),
    ct (CT_FLUX, or face-centred CT_FACE_AVG / CT_FACE_GS, whose face fields
    load_faces takes), integrator (INTEG_SSPRK2, INTEG_PC, INTEG_RK1, INTEG_SSPRK54),
    egrmhd (Extended GRMHD with the closure constants tau_r, chi_emhd,
    nu_emhd; needs INTEG_PC; its two extra variables via load_extended /
    extended).
    """

    def __init__(self, spec, gamma_ad, recon=RECON_WENO5, precision=PREC_FP64, cfl=0.9,
                 weno_eps=1e-26, newton_tol=1e-14, newton_maxit=30, device="cuda",
                 stream=None, strict=False, inverter=INV_1DW, kastaun_wmax=1e3, floors=False,
                 fofc=False, ct=CT_FLUX, integrator=INTEG_SSPRK2, egrmhd=False, tau_r=1.0,
                 chi_emhd=0.0, nu_emhd=0.0, **floor_params):
        self.spec = spec
        self.grid = make_grid(spec)
        self.metric = grmhd_metric(int(spec.metric), float(spec.a), float(spec.hslope))
        self.params = make_params(gamma_ad, cfl, weno_eps, newton_tol, newton_maxit, recon, precision,
                                  inverter, kastaun_wmax, floors, fofc, ct, integrator, egrmhd,
                                  tau_r, chi_emhd, nu_emhd, **floor_params)
        self.strict = strict
        L = lib()
        nbytes = L.grmhd_workspace_bytes(C.byref(self.grid), C.byref(self.params))
        if nbytes == 0:
            raise GrmhdError("invalid grid or parameters")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = (NVAR, spec.n3 + 2 * NG, spec.n2 + 2 * NG, spec.n1 + 2 * NG)
        ctx = C.c_void_p()
        _check(L.grmhd_create(C.byref(ctx), C.byref(self.grid), C.byref(self.metric),
                              C.byref(self.params), C.c_void_p(self._ws_ptr), nbytes,
                              C.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx
        self._lib = L
        _open.add(self)

    def close(self):
        """Release the context (idempotent); the object is unusable after."""
        ctx = getattr(self, "ctx", None)
        if ctx:
            self.ctx = None
            _open.discard(self)
            self._lib.grmhd_destroy(ctx)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may be gone when a late
        # finalizer runs)
        if not _finalizing():
            self.close()

    def load(self, prims):
        p = prims.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(p.shape) == self.shape, (p.shape, self.shape)
        self._keep = p
        _check(lib().grmhd_load_prims(self.ctx, _ptr(p)))

    def step(self, dt):
        _check(lib().grmhd_step(self.ctx, float(dt)))
        if self.strict and self.status()[0]:
            raise GrmhdError("inversion failures")

    def dt(self):
        out = C.c_double()
        _check(lib().grmhd_estimate_dt(self.ctx, C.byref(out)))
        return out.value

    def step_cfl(self):
        """One step at the CFL dt of the current state, reduced and used on
        the device (no host round trip); last_dt() reads it back."""
        _check(lib().grmhd_step_cfl(self.ctx))
        if self.strict and self.status()[0]:
            raise GrmhdError("inversion failures")

    def last_dt(self):
        out = C.c_double()
        _check(lib().grmhd_last_dt(self.ctx, C.byref(out)))
        return out.value

    def prims(self):
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(lib().grmhd_get_prims(self.ctx, _ptr(out)))
        return out

    def divb(self, field=False):
        mx, mean = C.c_double(), C.c_double()
        f = torch.zeros(self.shape[1:], dtype=torch.float64, device=self.device) if field else None
        _check(lib().grmhd_divb(self.ctx, _ptr(f), C.byref(mx), C.byref(mean)))
        return (mx.value, mean.value, f) if field else (mx.value, mean.value)

    def status(self):
        a, b = C.c_longlong(), C.c_longlong()
        _check(lib().grmhd_get_status(self.ctx, C.byref(a), C.byref(b)))
        return a.value, b.value

    def load_extended(self, extra):
        """Extended GRMHD's rescaled heat flux and pressure anisotropy,
        [2, n3+6, n2+6, n1+6] (zero after creation)."""
        x = extra.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(x.shape) == (2,) + tuple(self.shape[1:]), x.shape
        self._keep_extra = x
        _check(lib().grmhd_load_extended(self.ctx, _ptr(x)))

    def extended(self):
        out = torch.empty((2,) + tuple(self.shape[1:]), dtype=torch.float64, device=self.device)
        _check(lib().grmhd_get_extended(self.ctx, _ptr(out)))
        return out

    def load_faces(self, faces):
        """Face fields [3, n3+6, n2+6, n1+6] (sqrt(-g) B^d on lower d-faces) of
        face-centred CT."""
        f = faces.to(device=self.device, dtype=torch.float64).contiguous()
        assert tuple(f.shape) == (3,) + tuple(self.shape[1:])
        self._keep_faces = f
        _check(lib().grmhd_load_faces(self.ctx, _ptr(f)))

    def faces(self):
        out = torch.empty((3,) + tuple(self.shape[1:]), dtype=torch.float64, device=self.device)
        _check(lib().grmhd_get_faces(self.ctx, _ptr(out)))
        return out

    def face_divb(self):
        mx, mean = C.c_double(), C.c_double()
        _check(lib().grmhd_face_divb(self.ctx, C.byref(mx), C.byref(mean)))
        return mx.value, mean.value

    def counters(self):
        """Counts since creation or reset: failed inversions, zones floors
        acted on, zones the first-order flux correction marked, fluid-frame
        fallbacks of the floors."""
        out = (C.c_longlong * 4)()
        _check(lib().grmhd_get_counters(self.ctx, out))
        return dict(fails=out[0], floor_hits=out[1], fofc_zones=out[2], fluid_frame=out[3])

    def reset_status(self):
        _check(lib().grmhd_reset_status(self.ctx))

    def prims_to_cons(self, prims):
        p = prims.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.zeros_like(p)
        _check(lib().grmhd_prims_to_cons(self.ctx, _ptr(p), _ptr(out)))
        return out

    def cons_to_prims(self, cons, guess):
        u = cons.to(device=self.device, dtype=torch.float64).contiguous()
        g = guess.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.zeros_like(u)
        flags = torch.zeros(self.shape[1:], dtype=torch.int32, device=self.device)
        n = C.c_longlong()
        _check(lib().grmhd_cons_to_prims(self.ctx, _ptr(u), _ptr(g), _ptr(out), _ptr(flags),
                                         C.byref(n)))
        return out, n.value, flags

    def fluxes(self, prims):
        p = prims.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.zeros((3,) + self.shape, dtype=torch.float64, device=self.device)
        _check(lib().grmhd_fluxes(self.ctx, _ptr(p), _ptr(out)))
        return out

    TIMING_CLASSES = ("bc", "flux", "emf", "update1", "update2", "dt", "fofc", "floors", "faces")

    def step_vjp(self, prims_in, dt, gprims_out):
        """Adjoint of one step: (d loss/d prims_in, d loss/d gamma_ad)."""
        L = lib()
        if getattr(self, "_vjp_ws", None) is None:
            nb = L.grmhd_vjp_workspace_bytes(C.byref(self.grid), C.byref(self.params))
            if nb == 0:
                raise GrmhdError("invalid grid or parameters")
            self._vjp_ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            self._vjp_nb = nb
        off = (-self._vjp_ws.data_ptr()) % 256
        p = prims_in.to(device=self.device, dtype=torch.float64).contiguous()
        go = gprims_out.to(device=self.device, dtype=torch.float64).contiguous()
        gi = torch.empty_like(p)
        gg = C.c_double()
        _check(L.grmhd_step_vjp(self.ctx, _ptr(p), float(dt), _ptr(go), _ptr(gi), C.byref(gg),
                                C.c_void_p(self._vjp_ws.data_ptr() + off), self._vjp_nb))
        return gi, gg.value

    def set_schedule(self, kg_flux, kg_update):
        _check(lib().grmhd_set_schedule(self.ctx, int(kg_flux), int(kg_update)))

    def timing(self, enable=True, classes=None):
        """Per-launch timing events on (all classes, or the named ones) or off."""
        if not enable:
            mask = 0
        elif classes is None:
            mask = -1
        else:
            mask = sum(1 << self.TIMING_CLASSES.index(k) for k in classes)
        _check(lib().grmhd_timing(self.ctx, int(mask)))

    def timing_report(self):
        n = len(self.TIMING_CLASSES)
        ms = (C.c_double * n)()
        cnt = (C.c_longlong * n)()
        _check(lib().grmhd_timing_report(self.ctx, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.TIMING_CLASSES)}


class Pack:
    """A pack of cubic blocks (sub-boxes of one global grid) advanced together
    by three launches per RK2 stage (fluxes, EMFs, update) over all blocks."""

    def __init__(self, global_spec, sizes, offsets, gamma_ad, recon=RECON_WENO5, cfl=0.9,
                 weno_eps=1e-26, newton_tol=1e-14, newton_maxit=30, device="cuda", stream=None,
                 inverter=INV_1DW, kastaun_wmax=1e3):
        L = lib()
        self.nb = len(sizes)
        self.sizes = [int(n) for n in sizes]
        self._n = (C.c_int * self.nb)(*self.sizes)
        flat = [int(v) for o in offsets for v in o]
        self._off = (C.c_int * (3 * self.nb))(*flat)
        self.grid = make_grid(global_spec)
        self.metric = grmhd_metric(int(global_spec.metric), float(global_spec.a),
                                   float(global_spec.hslope))
        self.params = make_params(gamma_ad, cfl, weno_eps, newton_tol, newton_maxit, recon, PREC_FP64,
                                  inverter, kastaun_wmax)
        nbytes = L.grmhd_pack_workspace_bytes(self.nb, self._n)
        if nbytes == 0:
            raise GrmhdError("invalid pack")
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(L.grmhd_pack_create(C.byref(h), self.nb, self._n, self._off, C.byref(self.grid),
                                   C.byref(self.metric), C.byref(self.params),
                                   C.c_void_p(self.workspace.data_ptr() + off), nbytes,
                                   C.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self._lib = L
        _open.add(self)
        gb, nd = C.c_int(), C.c_longlong()
        _check(L.grmhd_pack_info(self.h, C.byref(gb), C.byref(nd)))
        self.grid_blocks, self.prim_doubles = gb.value, nd.value

    def close(self):
        """Release the pack (idempotent); the object is unusable after."""
        h = getattr(self, "h", None)
        if h:
            self.h = None
            _open.discard(self)
            self._lib.grmhd_pack_destroy(h)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may be gone when a late
        # finalizer runs)
        if not _finalizing():
            self.close()

    def set_tiles(self, n, t1, t2, t3):
        _check(lib().grmhd_pack_set_tiles(self.h, int(n), int(t1), int(t2), int(t3)))

    def set_exchange(self, on=True):
        """Ghost exchange between the blocks before every stage (on), or
        frozen ghosts (off, the default); the owner map lives in a tensor
        kept here."""
        L = lib()
        if not on:
            _check(L.grmhd_pack_set_exchange(self.h, None, 0))
            self._owner = None
            return
        nbytes = L.grmhd_pack_exchange_bytes(C.byref(self.grid))
        self._owner = torch.empty(nbytes // 4, dtype=torch.int32, device=self.device)
        _check(L.grmhd_pack_set_exchange(self.h, _ptr(self._owner), nbytes))

    def load(self, packed):
        p = packed.to(device=self.device, dtype=torch.float64).contiguous()
        assert p.numel() == self.prim_doubles
        self._keep = p
        _check(lib().grmhd_pack_load_prims(self.h, _ptr(p)))

    def step(self, dt):
        _check(lib().grmhd_pack_step(self.h, float(dt)))

    def prims(self):
        out = torch.empty(self.prim_doubles, dtype=torch.float64, device=self.device)
        _check(lib().grmhd_pack_get_prims(self.h, _ptr(out)))
        return out

    def status(self):
        n = C.c_longlong()
        _check(lib().grmhd_pack_get_status(self.h, C.byref(n)))
        return n.value
