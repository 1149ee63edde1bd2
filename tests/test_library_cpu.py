"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, validates arguments and sizes its
workspace."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "grmhd.h")).read()
    return sorted(set(re.findall(r"\b(grmhd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2408_01361_amd import grmhd
    lib = grmhd.lib()
    names = _header_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(grmhd.EXPORTS)


def test_workspace_and_argument_validation():
    from paper_2408_01361_amd import grmhd
    from workloads import GridSpec, torus_grid
    lib = grmhd.lib()
    p = grmhd.grmhd_params(13 / 9, 0.9, 1e-26, 1e-14, 30, grmhd.RECON_WENO5, grmhd.PREC_FP64, 0)
    g = grmhd.make_grid(torus_grid(128, 128, 128))
    nb = lib.grmhd_workspace_bytes(C.byref(g), C.byref(p))
    nz = 134 ** 3
    assert nb >= 8 * nz * 8 * 6          # state, stage, V and three flux arrays
    assert nb < 8 * nz * 8 * 8
    bad = grmhd.make_grid(torus_grid(128, 2, 128))   # polar axis needs >= 3 zones
    assert lib.grmhd_workspace_bytes(C.byref(bad), C.byref(p)) == 0
    p2 = grmhd.grmhd_params(13 / 9, 0.9, 1e-26, 1e-14, 30, 8, grmhd.PREC_FP64, 0)
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(p2)) == 0
    p3 = grmhd.grmhd_params(13 / 9, 0.9, 1e-26, 1e-14, 30, 0, grmhd.PREC_FP64, 1)
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(p3)) == 0
    # the Kastaun recovery needs a Lorentz-factor cap above 1; 1D_W ignores it
    pk = grmhd.grmhd_params(13 / 9, 0.9, 1e-26, 1e-14, 30, 0, grmhd.PREC_FP64, 0,
                            grmhd.INV_KASTAUN, 1e3)
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(pk)) == nb
    pk.kastaun_wmax = 1.0
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(pk)) == 0
    pk.inverter = 3
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(pk)) == 0
    # a null workspace is rejected before any device call
    ctx = C.c_void_p()
    m = grmhd.grmhd_metric(1, 0.9375, 0.3)
    assert lib.grmhd_create(C.byref(ctx), C.byref(g), C.byref(m), C.byref(p), None, nb, None) == grmhd.E_ARG
    assert lib.grmhd_step(None, 0.1) == grmhd.E_ARG
    assert lib.grmhd_strerror(grmhd.E_NOMEM) == b"workspace too small"


def test_floor_and_correction_parameters_are_validated():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(32, 32, 32))
    mk = lambda **kw: grmhd.make_params(13 / 9, 0.9, 1e-26, 1e-14, 30, grmhd.RECON_WENO5,
                                        grmhd.PREC_FP64, 0, 1e3, **kw)
    ok = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(floors=True, fofc=True)))
    assert ok > 0
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(floors=True, gamma_max=1.0))) == 0
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(floors=True, rho_min_geom=0.0))) == 0
    # parameters of disabled floors are not looked at
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(floors=False, gamma_max=0.0))) > 0
    p = mk(fofc=True)
    p.fofc = 2
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(p)) == 0
    # the adjoint covers the plain high-order step only
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(fofc=True))) == 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(floors=True))) == 0
    donor = grmhd.make_params(13 / 9, 0.9, 1e-26, 1e-14, 30, grmhd.RECON_DONOR, grmhd.PREC_FP64, 0, 1e3)
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(donor)) > 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(donor)) == 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk())) > 0


def test_reconstruction_choices_are_validated():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(32, 32, 32))
    mk = lambda recon, eps=1e-26: grmhd.make_params(13 / 9, 0.9, eps, 1e-14, 30, recon,
                                                     grmhd.PREC_FP64, 0, 1e3)
    base = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(grmhd.RECON_WENO5)))
    for r in (grmhd.RECON_MC, grmhd.RECON_DONOR, grmhd.RECON_WENOZ, grmhd.RECON_VL, grmhd.RECON_MP5,
              grmhd.RECON_PPM, grmhd.RECON_PPMX):
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(r))) == base
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(8))) == 0
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(-1))) == 0
    # the WENO regulariser must keep the weight products normal ...
    for r in (grmhd.RECON_WENO5, grmhd.RECON_WENOZ):
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(r, 1e-40))) == 0
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(r, 2.0))) == 0
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(r, 1e-36))) == base
    # ... and is not looked at by the other schemes
    for r in (grmhd.RECON_VL, grmhd.RECON_MP5, grmhd.RECON_PPM, grmhd.RECON_PPMX):
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(r, 0.0))) == base
    # the adjoint and packs take MC or WENO5 only
    for r in (grmhd.RECON_WENOZ, grmhd.RECON_VL, grmhd.RECON_MP5, grmhd.RECON_PPM, grmhd.RECON_PPMX):
        assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(r))) == 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(grmhd.RECON_MC))) > 0


def test_integrator_parameters_are_validated():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(32, 32, 32))
    mk = lambda integ, **kw: grmhd.make_params(13 / 9, 0.9, 1e-26, 1e-14, 30, grmhd.RECON_WENO5,
                                               grmhd.PREC_FP64, 0, 1e3, integrator=integ, **kw)
    base = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(grmhd.INTEG_SSPRK2)))
    nz = 38 ** 3
    for integ in (grmhd.INTEG_PC, grmhd.INTEG_RK1, grmhd.INTEG_SSPRK54):
        # SSPRK(5,4) keeps two more conserved-variable registers
        extra = 2 * 8 * nz * 8 if integ == grmhd.INTEG_SSPRK54 else 0
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(integ))) == base + extra
        # the other integrators take the plain Flux-CT step only
        for kw in (dict(floors=True), dict(fofc=True), dict(ct=grmhd.CT_FACE_GS)):
            assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(integ, **kw))) == 0
        assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(integ))) == 0
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(4))) == 0
    p = mk(grmhd.INTEG_PC)
    p.inverter = grmhd.INV_IMPLICIT
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(p)) == 0


def test_pack_exchange_map_size():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(64, 48, 32))
    assert lib.grmhd_pack_exchange_bytes(C.byref(g)) == 4 * 64 * 48 * 32
    assert lib.grmhd_pack_set_exchange(None, None, 0) == grmhd.E_ARG


def test_face_ct_parameters_and_workspace():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(32, 32, 32))
    mk = lambda **kw: grmhd.make_params(13 / 9, 0.9, 1e-26, 1e-14, 30, grmhd.RECON_WENO5,
                                        grmhd.PREC_FP64, 0, 1e3, **kw)
    base = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk()))
    face = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(ct=grmhd.CT_FACE_GS)))
    nz = 38 ** 3
    assert face >= base + 13 * 8 * nz          # faces, stage faces, register, zone EMFs, mass-current scale
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(ct=3))) == 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(ct=grmhd.CT_FACE_AVG))) == 0
    assert lib.grmhd_load_faces(None, None) == grmhd.E_ARG


def test_implicit_recovery_parameters():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(32, 32, 32))
    mk = lambda inv, **kw: grmhd.make_params(13 / 9, 0.9, 1e-26, 1e-14, 30, grmhd.RECON_WENO5,
                                             grmhd.PREC_FP64, inv, 1e3, **kw)
    base = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(0)))
    impl = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(grmhd.INV_IMPLICIT)))
    assert impl >= base + 8 * 8 * 38 ** 3          # the stored U* of a stage
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(grmhd.INV_IMPLICIT, fofc=True))) == 0
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(4))) == 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(grmhd.INV_IMPLICIT))) == 0


def test_extended_grmhd_parameters_and_workspace():
    from paper_2408_01361_amd import grmhd
    from workloads import torus_grid
    lib = grmhd.lib()
    g = grmhd.make_grid(torus_grid(32, 32, 32))
    mk = lambda **kw: grmhd.make_params(13 / 9, 0.9, 1e-26, 1e-14, 30, kw.pop("recon", grmhd.RECON_WENO5),
                                        kw.pop("precision", grmhd.PREC_FP64), 0, 1e3,
                                        **{"integrator": grmhd.INTEG_PC, **kw})
    base = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk()))
    ext = lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(egrmhd=True, tau_r=1.0, chi_emhd=0.1, nu_emhd=0.1)))
    nz = 38 ** 3
    # U* of a stage; the state's and stage 1's X, their fluxes, U^n and
    # right-hand sides of X; u^t of the step start and the spatial div u
    assert ext >= base + (8 + 2 * 7 + 2) * 8 * nz
    for mc in (grmhd.RECON_MC, grmhd.RECON_WENO5):
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(egrmhd=True, recon=mc))) > 0
    bad = [dict(egrmhd=True, integrator=grmhd.INTEG_SSPRK2), dict(egrmhd=True, integrator=grmhd.INTEG_RK1),
           dict(egrmhd=True, precision=grmhd.PREC_MIXED), dict(egrmhd=True, recon=grmhd.RECON_MP5),
           dict(egrmhd=True, tau_r=0.0), dict(egrmhd=True, tau_r=float("nan")),
           dict(egrmhd=True, chi_emhd=-1.0), dict(egrmhd=True, nu_emhd=float("inf"))]
    for kw in bad:
        assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(mk(**kw))) == 0, kw
    p = mk(egrmhd=True)
    p.egrmhd = 2
    assert lib.grmhd_workspace_bytes(C.byref(g), C.byref(p)) == 0
    assert lib.grmhd_vjp_workspace_bytes(C.byref(g), C.byref(mk(egrmhd=True))) == 0
    assert lib.grmhd_load_extended(None, None) == grmhd.E_ARG
    assert lib.grmhd_get_extended(None, None) == grmhd.E_ARG
