"""GPU-vs-oracle parity at the full workload sizes, in the launch
configuration bench.py times (default schedule, device-side CFL step), and
at the edges of the parameter space: one-zone axes, ragged sizes, and a grid
larger than one reduction partial per workgroup.

The oracle runs whole steps here (OpenMP over x3 planes), so every zone is
compared, to the same bars as the small cases (parity_util.check: relative
L1 per primitive at most 1e-12 per step, every zone within the per-zone
bars), failure counts equal.
"""

import os

import numpy as np
import pytest

import oracle
from parity_util import GROUPS, rel_l1, check, zone_rel, ZONE_TOL
from workloads import (GridSpec, fm_torus, interior, linear_mode, torus_pack, BC_PERIODIC,
                       METRIC_MINKOWSKI, RECON_MC, RECON_WENO5)

pytestmark = pytest.mark.gpu

TOL = 1e-12
THREADS = min(16, os.cpu_count() or 1)


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01361_amd import grmhd as gr
    return torch, gr


def test_torus128_weno5_full_step_as_benchmarked():
    """The benchmark workload itself: 128^3 magnetised torus, WENO5, FP64, one
    device-side CFL step; dt and every zone against the oracle."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5)
    s.load(torch.from_numpy(P).cuda())
    s.step_cfl()
    dt = s.last_dt()
    out = s.prims().cpu().numpy()
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS)
    assert dt == pytest.approx(oracle.estimate_dt(c, P), rel=1e-14)
    ref, fails, _ = oracle.run(c, P, dt, 1)
    print("128^3 WENO5 failures", fails)
    check(out, ref, label="128^3 WENO5")
    assert s.status()[0] == fails


def test_torus128_weno5_kastaun_full_step():
    """The benchmark workload with the Kastaun et al. recovery in place of
    1D_W: one device-side CFL step, every zone against the oracle."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5, inverter=gr.INV_KASTAUN)
    s.load(torch.from_numpy(P).cuda())
    s.step_cfl()
    dt = s.last_dt()
    out = s.prims().cpu().numpy()
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS, inverter=oracle.INV_KASTAUN)
    ref, fails, _ = oracle.run(c, P, dt, 1)
    print("128^3 WENO5 Kastaun failures", fails)
    check(out, ref, label="128^3 WENO5 Kastaun")
    assert s.status()[0] == fails


def test_torus128_weno5_implicit_recovery_full_step():
    """The benchmark workload with the implicit solver's Newton as the
    recovery: one device-side CFL step, every zone against the oracle."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5, inverter=gr.INV_IMPLICIT)
    s.load(torch.from_numpy(P).cuda())
    s.step_cfl()
    dt = s.last_dt()
    out = s.prims().cpu().numpy()
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS, inverter=oracle.INV_IMPLICIT)
    ref, fails, _ = oracle.run(c, P, dt, 1)
    print("128^3 WENO5 implicit recovery failures", fails)
    check(out, ref, label="128^3 WENO5 implicit")
    assert s.status()[0] == fails


def test_torus128_weno5_face_ct_full_step():
    """The benchmark workload with face-centred CT (upwinded EMFs): one step
    at the oracle's dt, every zone and every evolved face against the
    oracle; face divergence at roundoff."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, info = fm_torus(128, 128, 128, seed=1, gamma=gam)
    F = info["faces"]
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS, ct=oracle.CT_FACE_GS)
    ref, Fref, fails, dts = oracle.run_face(c, P, F, -1, 1)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5, ct=gr.CT_FACE_GS)
    s.load(torch.from_numpy(P).cuda())
    s.load_faces(torch.from_numpy(F).cuda())
    s.step(float(dts[0]))
    out, Fo = s.prims().cpu().numpy(), s.faces().cpu().numpy()
    A, B = Fo[:, 3:-2, 3:-2, 3:-2], Fref[:, 3:-2, 3:-2, 3:-2]
    rf = np.abs(A - B).sum() / np.abs(B).sum()
    print("128^3 face-CT faces", rf, "failures", fails)
    check(out, ref, label="128^3 face-CT")
    assert rf <= TOL
    assert s.status()[0] == fails
    assert s.face_divb()[0] < 1e-13 * np.abs(F).max() / min(grid.dx)


def test_torus192_fp64_full_step():
    """The reduced-precision workload's grid in FP64 (the reference its error
    is stated against): 192^3, WENO5, one step."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(192, 192, 192, seed=1, gamma=gam)
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS)
    dt = oracle.estimate_dt(c, P)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5)
    s.load(torch.from_numpy(P).cuda())
    s.step(dt)
    out = s.prims().cpu().numpy()
    ref, fails, _ = oracle.run(c, P, dt, 1)
    check(out, ref, label="192^3 WENO5")
    assert s.status()[0] == fails


def test_full_pack_320_blocks_against_oracle():
    """The batched workload: all 320 blocks, one pack step against the oracle
    block by block (relative L1 over the whole pack)."""
    torch, gr = _setup()
    gam = 13 / 9
    g, blocks, _ = torus_pack(nblocks=320, n_global=128, sizes=(16, 32, 64), probs=(0.6, 0.3, 0.1),
                              seed=7, torus_seed=1, gamma=gam)
    _, Pg, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    dt = oracle.estimate_dt(oracle.cfg(g, gam=gam, recon=RECON_WENO5, nthreads=THREADS), Pg)
    pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], gam, recon=RECON_WENO5)
    pk.load(torch.from_numpy(np.concatenate([b["prims"].ravel() for b in blocks])).cuda())
    pk.step(dt)
    flat = pk.prims().cpu().numpy()
    num, den, o, fails = np.zeros(8), np.zeros(8), 0, 0
    zone = np.zeros(8)
    for b in blocks:
        n = b["n"] + 6
        out = flat[o:o + 8 * n ** 3].reshape(8, n, n, n)
        o += 8 * n ** 3
        ref, f, _ = oracle.run(oracle.cfg(b["grid"], gam=gam, recon=RECON_WENO5, nthreads=THREADS),
                               b["prims"], dt, 1)
        fails += f
        zone = np.maximum(zone, zone_rel(out, ref))
        A, B = interior(out), interior(ref)
        for v in range(8):
            num[v] += np.abs(A[v] - B[v]).sum()
            den[v] += sum(np.abs(B[w]).sum() for w in GROUPS[v])
    rel = num / den
    print("pack rel L1", rel, "per zone", zone, "failures", fails, pk.status())
    assert rel.max() <= TOL, rel
    assert np.all(zone <= ZONE_TOL), zone
    assert pk.status() == fails


@pytest.mark.parametrize("shape,recon", [((37, 1, 1), RECON_WENO5), ((1, 29, 1), RECON_MC),
                                         ((1, 1, 23), RECON_WENO5), ((17, 13, 5), RECON_MC),
                                         ((19, 3, 7), RECON_WENO5)])
def test_one_zone_axes_and_ragged_sizes(shape, recon):
    """Grids with one-zone axes (the step is then 1-D or 2-D) and sizes that
    fill no tile or wavefront evenly; a seeded random smooth state in flat
    space with all eight primitives varying."""
    torch, gr = _setup()
    n1, n2, n3 = shape
    grid = GridSpec(n1, n2, n3, bc=(BC_PERIODIC,) * 6, metric=METRIC_MINKOWSKI)
    x1, x2, x3 = grid.centers()
    X3, X2, X1 = np.meshgrid(x3, x2, x1, indexing="ij")
    rng = np.random.default_rng(sum(shape))
    base = np.array([1.0, 1.0, 0.1, -0.2, 0.15, 0.8, 0.3, -0.4])
    P = np.empty((8,) + X1.shape)
    for v in range(8):
        a, ph = rng.uniform(0.05, 0.2, 3), rng.uniform(0, 2 * np.pi, 3)
        P[v] = base[v] * (1 + 0.0) + a[0] * np.sin(2 * np.pi * X1 + ph[0]) \
            + a[1] * np.sin(2 * np.pi * X2 + ph[1]) + a[2] * np.sin(2 * np.pi * X3 + ph[2])
    P[0] = np.abs(P[0]) + 0.5
    P[1] = np.abs(P[1]) + 0.5
    c = oracle.cfg(grid, gam=4 / 3, recon=recon)
    dt = oracle.estimate_dt(c, P)
    ref, fails, _ = oracle.run(c, P, dt, 2)
    s = gr.Grmhd(grid, 4 / 3, recon=recon)
    s.load(torch.from_numpy(P).cuda())
    s.step(dt)
    s.step(dt)
    out = s.prims().cpu().numpy()
    assert fails == 0 and s.status()[0] == 0
    check(out, ref, label=str(shape))
    # the random field is not divergence-free; Flux-CT keeps its corner
    # divergence unchanged to roundoff
    mx, mean = s.divb()
    mx0, mean0 = oracle.divb(c, P)
    assert mx == pytest.approx(mx0, rel=1e-9) and mean == pytest.approx(mean0, rel=1e-9)


def test_large_grid_256():
    """256^3 torus (16.8 M zones: more interior zones than reduction
    partials of one zone per thread), WENO5, one step, every zone."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(256, 256, 256, seed=1, gamma=gam)
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5)
    s.load(torch.from_numpy(P).cuda())
    dt = s.dt()
    assert dt == pytest.approx(oracle.estimate_dt(c, P), rel=1e-14)
    s.step(dt)
    out = s.prims().cpu().numpy()
    ref, fails, _ = oracle.run(c, P, dt, 1)
    print("256^3 failures", fails)
    check(out, ref, label="256^3")
    assert s.status()[0] == fails


def test_mixed_precision_192_against_oracle():
    """The reduced-precision workload (192^3 torus, WENO5, FP32 fluxes and
    EMFs) against the FP64 oracle after one step: the stated density error
    (about 7e-10 relative L1) and div B at roundoff (the CT update is FP64)."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(192, 192, 192, seed=1, gamma=gam)
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, nthreads=THREADS)
    dt = oracle.estimate_dt(c, P)
    s = gr.Grmhd(grid, gam, recon=RECON_WENO5, precision=gr.PREC_MIXED)
    s.load(torch.from_numpy(P).cuda())
    s.step(dt)
    out = s.prims().cpu().numpy()
    ref, _, _ = oracle.run(c, P, dt, 1)
    rho = np.abs(interior(out)[0] - interior(ref)[0]).sum() / np.abs(interior(ref)[0]).sum()
    rel = rel_l1(out, ref)
    print("mixed 192^3 vs oracle: rho rel L1", rho, "per variable", rel)
    assert rho < 5e-9
    mx, _ = s.divb()
    assert mx < 1e-13 * np.abs(interior(P[5:8])).max() / grid.dx[0]
