"""GPU-vs-oracle parity of face-centred constrained transport (averaged and
upwinded edge EMFs), through the C ABI.

Both sides advance the same prims and face fields (sqrt(-g) B^d on lower
faces) with the oracle's dt; the bar is the step bar (relative L1 of every
primitive at most 1e-12 per step) and the same for the evolved faces
(relative to the L1 norm of all three face families); ghost faces equal the
oracle's bit for bit; the face divergence stays at roundoff on the GPU."""

import numpy as np
import pytest

import oracle
from parity_util import rel_l1, check, NOISY_MODE
from workloads import (magnetised_blast, fm_torus, linear_mode_faces, interior, RECON_MC, RECON_WENO5)

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01361_amd import grmhd as gr
    return torch, gr


def faces_rel_l1(a, b):
    """Relative L1 of the evolved faces (interior zones' lower faces plus the
    upper boundary faces) against the L1 norm of all three families."""
    A, B = a[:, 3:-2, 3:-2, 3:-2], b[:, 3:-2, 3:-2, 3:-2]
    den = np.abs(B).sum()
    return np.abs(A - B).sum() / den if den > 0 else np.abs(A - B).max()


def run_both(grid, P, F, gam, recon, ct, nsteps, noisy=(), **kw):
    torch, gr = _setup()
    c = oracle.cfg(grid, gam=gam, recon=recon, ct=ct, **kw)
    alt, _, _, _ = oracle.run_face(c, P, F, -1, nsteps, fma=True)
    ref, Fref, fails, dts = oracle.run_face(c, P, F, -1, nsteps)
    st = oracle.last_stats()
    spread = rel_l1(alt, ref)
    run_both.alt = alt
    s = gr.Grmhd(grid, gam, recon=recon, ct=ct, **kw)
    s.load(torch.from_numpy(P).cuda())
    s.load_faces(torch.from_numpy(F).cuda())
    for dt in dts:
        s.step(float(dt))
    return s.prims().cpu().numpy(), s.faces().cpu().numpy(), ref, Fref, s, st, c, spread


def _mode(ct, recon):
    g, P, F, _, _ = linear_mode_faces("fast", 32, ndim=2)
    return g, P, F, 4 / 3, recon


def _torus(n1, n2, n3):
    grid, P, info = fm_torus(n1, n2, n3)
    return grid, P, info["faces"], 13 / 9


CASES = {
    "fast32_mc_avg": (lambda: _mode(1, RECON_MC), 1, 2, dict(noisy=NOISY_MODE)),
    "fast32_mc_gs": (lambda: _mode(2, RECON_MC), 2, 2, dict(noisy=NOISY_MODE)),
    "fast32_weno_gs": (lambda: _mode(2, RECON_WENO5), 2, 2, dict(noisy=NOISY_MODE)),
    "torus24_weno_gs": (lambda: _torus(24, 24, 8) + (RECON_WENO5,), 2, 2, {}),
    "torus20x28x6_mc_avg": (lambda: _torus(20, 28, 6) + (RECON_MC,), 1, 2, {}),
    "blast48_mc_gs_floors_fofc": (lambda: magnetised_blast(48, faces=True) + (4 / 3, RECON_MC), 2, 4,
                                  dict(floors=True, fofc=True)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_face_ct_parity(case):
    make, ct, nsteps, kw = CASES[case]
    kw = dict(kw)
    noisy = kw.pop("noisy", ())
    grid, P, F, gam, recon = make()
    out, Fo, ref, Fref, s, st, c, spread = run_both(grid, P, F, gam, recon, ct, nsteps, noisy, **kw)
    rf = faces_rel_l1(Fo, Fref)
    cnt = s.counters()
    print(case, "faces", rf, "gpu", cnt, "oracle", st, "oracle FMA spread", spread, flush=True)
    assert cnt == st
    check(out, ref, noisy, spread, label=case, alt=run_both.alt)
    assert rf <= TOL, rf
    mx, _ = s.face_divb()
    omx, _ = oracle.face_divb(c, Fref)
    scale = np.abs(F).max() / min(grid.dx)
    assert mx < 1e-13 * scale and omx < 1e-13 * scale, (mx, omx)


@pytest.mark.parametrize("which", ["mode", "torus"])
def test_ghost_faces_match_the_oracle(which):
    """Loaded faces come back with ghost faces equal to the oracle's fill
    (periodic; outflow, polar mirror with the normal sign flip, periodic)
    bit for bit, and the zone B set to the faces' mean."""
    torch, gr = _setup()
    if which == "mode":
        grid, P, F, gam, recon = _mode(2, RECON_MC)
    else:
        grid, P, F, gam = _torus(20, 24, 6)
        recon = RECON_MC
    c = oracle.cfg(grid, gam=gam, recon=recon, ct=2)
    Pref, Fref, _, _ = oracle.run_face(c, P, F, 1e-30, 0)
    s = gr.Grmhd(grid, gam, recon=recon, ct=2)
    s.load(torch.from_numpy(P).cuda())
    s.load_faces(torch.from_numpy(F).cuda())
    Fo = s.faces().cpu().numpy()
    assert np.array_equal(Fo, Fref)
    Po = s.prims().cpu().numpy()
    assert np.abs(interior(Po)[5:8] - interior(Pref)[5:8]).max() <= 1e-15 * np.abs(interior(Pref)[5:8]).max()


def test_face_ct_cfl_steps_and_mixed_precision():
    """Device CFL steps with face-centred CT; the reduced-precision path
    (FP32 fluxes and EMFs, FP64 faces) keeps the face divergence at FP64
    roundoff; with averaged EMFs its density error against FP64 is of the
    size of the Flux-CT path's (measured beside it, same steps at the same
    dt).  The upwinded EMFs switch on the sign of the face mass flux, which
    FP32 decides differently from FP64 where that flux is physically small:
    their error is stated, bounded at 1e-4 here."""
    torch, gr = _setup()
    grid, P, F, gam = _torus(32, 32, 16)
    res = {}
    dt = None
    for ct in (0, 1, 2):
        for prec in (gr.PREC_FP64, gr.PREC_MIXED):
            s = gr.Grmhd(grid, gam, recon=RECON_WENO5, ct=ct, precision=prec)
            s.load(torch.from_numpy(P).cuda())
            if ct:
                s.load_faces(torch.from_numpy(F).cuda())
            dt = dt or s.dt()
            for _ in range(4):
                s.step(dt)
            res[ct, prec] = (s.prims().cpu().numpy(), s.face_divb()[0] if ct else 0.0, s)
    scale = np.abs(F).max() / min(grid.dx)
    err = {}
    for ct in (0, 1, 2):
        a, b = interior(res[ct, gr.PREC_FP64][0])[0], interior(res[ct, gr.PREC_MIXED][0])[0]
        err[ct] = np.abs(a - b).sum() / np.abs(a).sum()
    print("mixed vs FP64 density rel L1: Flux-CT", err[0], "face-CT averaged", err[1], "upwinded", err[2],
          "face div", res[2, gr.PREC_FP64][1], res[2, gr.PREC_MIXED][1])
    for ct in (1, 2):
        assert res[ct, gr.PREC_FP64][1] < 1e-13 * scale and res[ct, gr.PREC_MIXED][1] < 1e-13 * scale
    assert err[1] < 10 * err[0] + 1e-9
    assert err[2] < 1e-4
    sa = res[2, gr.PREC_FP64][2]
    a = res[2, gr.PREC_FP64][0]
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, ct=2)
    sa.step_cfl()
    assert sa.last_dt() == pytest.approx(oracle.estimate_dt(c, a), rel=1e-14)


def test_face_ct_requires_faces():
    torch, gr = _setup()
    grid, P, F, gam = _torus(16, 16, 4)
    s = gr.Grmhd(grid, gam, recon=RECON_MC, ct=2)
    s.load(torch.from_numpy(P).cuda())
    with pytest.raises(gr.GrmhdError):
        s.step(0.1)


@pytest.mark.parametrize("ct", [1, 2])
def test_face_ct_keeps_the_torus_symmetries_on_the_gpu(ct):
    """The unperturbed magnetised torus with face-centred CT on the GPU:
    identical x3 slices bit for bit, equatorial mirror symmetry (u~2 flipped,
    B -> (-B1, B2, -B3)) to roundoff."""
    torch, gr = _setup()
    grid, P, info = fm_torus(48, 48, 4, noise=0.0, magnetised=True)
    s = gr.Grmhd(grid, 13 / 9, recon=RECON_WENO5, ct=ct)
    s.load(torch.from_numpy(P).cuda())
    s.load_faces(torch.from_numpy(info["faces"]).cuda())
    dt = s.dt()
    for _ in range(2):
        s.step(dt)
    I = interior(s.prims().cpu().numpy())
    for k in range(1, 4):
        assert np.array_equal(I[:, k], I[:, 0])
    M = I[:, :, ::-1, :].copy()
    M[3] *= -1
    M[5] *= -1
    M[7] *= -1
    scale = np.abs(I).max(axis=(1, 2, 3))[:, None, None, None] + 1e-300
    err = (np.abs(M - I) / scale).max()
    print("mirror error", err)
    assert err < 1e-11
