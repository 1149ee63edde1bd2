"""GPU-vs-oracle parity of the further reconstructions: WENO-Z (power 2),
linear reconstruction with van Leer's limiter, MP5, PPM and PPMX, through
the C ABI.

Bars as for MC and WENO5 (parity_util.check): relative L1 per primitive at
most 1e-12 per step, every zone within the per-zone bars, failure counts
equal; the u~ of a linear mode at rest (its whole value the perturbation) is
held to 3x the oracle's own FMA spread on the case, since the GPU's face
physics rounds differently from the oracle's written form.  The
mixed-precision forms are held against the FP64 GPU path of the same
reconstruction.
"""

import os

import numpy as np
import pytest

import oracle
from parity_util import rel_l1, check, zone_rel, ZONE_TOL, NOISY_MODE
from workloads import linear_mode, fm_torus, bondi, interior, torus_pack

pytestmark = pytest.mark.gpu

TOL = 1e-12
THREADS = min(16, os.cpu_count() or 1)
WENOZ, VL, MP5, PPM, PPMX = (oracle.RECON_WENOZ, oracle.RECON_VL, oracle.RECON_MP5, oracle.RECON_PPM,
                             oracle.RECON_PPMX)


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01361_amd import grmhd as gr
    return torch, gr


# case: ((grid, prims), gamma, reconstruction, noisy components)
CASES = {
    "fast16_wenoz": lambda: (linear_mode("fast", 16, ndim=3)[0:2], 4 / 3, WENOZ, NOISY_MODE),
    "torus24_wenoz": lambda: (fm_torus(24, 24, 8)[0:2], 13 / 9, WENOZ, ()),
    "bondi24x12x2_wenoz": lambda: (bondi(24, 12, 2)[0:2], 4 / 3, WENOZ, ()),
    "fast32_vl": lambda: (linear_mode("fast", 32, ndim=3)[0:2], 4 / 3, VL, NOISY_MODE),
    "alfven24x20_vl_2d": lambda: (linear_mode("alfven", 24, ndim=2)[0:2], 4 / 3, VL, NOISY_MODE),
    "torus20x28x6_vl": lambda: (fm_torus(20, 28, 6)[0:2], 13 / 9, VL, ()),
    "bondi32x16_vl": lambda: (bondi(32, 16)[0:2], 4 / 3, VL, ()),
    "fast16_mp5": lambda: (linear_mode("fast", 16, ndim=3)[0:2], 4 / 3, MP5, NOISY_MODE),
    "slow20_mp5_2d": lambda: (linear_mode("slow", 20, ndim=2)[0:2], 4 / 3, MP5, NOISY_MODE),
    "torus24_mp5": lambda: (fm_torus(24, 24, 8)[0:2], 13 / 9, MP5, ()),
    "bondi24x12x2_mp5": lambda: (bondi(24, 12, 2)[0:2], 4 / 3, MP5, ()),
    "fast16_ppm": lambda: (linear_mode("fast", 16, ndim=3)[0:2], 4 / 3, PPM, NOISY_MODE),
    "alfven24x20_ppm_2d": lambda: (linear_mode("alfven", 24, ndim=2)[0:2], 4 / 3, PPM, NOISY_MODE),
    "torus20x28x6_ppm": lambda: (fm_torus(20, 28, 6)[0:2], 13 / 9, PPM, ()),
    "bondi32x16_ppm": lambda: (bondi(32, 16)[0:2], 4 / 3, PPM, ()),
    "fast16_ppmx": lambda: (linear_mode("fast", 16, ndim=3)[0:2], 4 / 3, PPMX, NOISY_MODE),
    "alfven24x20_ppmx_2d": lambda: (linear_mode("alfven", 24, ndim=2)[0:2], 4 / 3, PPMX, NOISY_MODE),
    "torus20x28x6_ppmx": lambda: (fm_torus(20, 28, 6)[0:2], 13 / 9, PPMX, ()),
    "bondi32x16_ppmx": lambda: (bondi(32, 16)[0:2], 4 / 3, PPMX, ()),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_step_parity_further_reconstructions(case):
    torch, gr = _setup()
    (grid, P), gam, recon, noisy = CASES[case]()
    print("case", case, flush=True)
    c = oracle.cfg(grid, gam=gam, recon=recon)
    ref, fails, dts, _ = oracle.run(c, P, -1, 2, flags=True)
    alt = oracle.run(c, P, -1, 2, fma=True)[0] if noisy else None
    s = gr.Grmhd(grid, gam, recon=recon)
    s.load(torch.from_numpy(P))
    for dt in dts:
        s.step(dt)
    out = s.prims().cpu().numpy()
    print(case, "dts", dts, "fails", fails, s.status()[0], )
    assert s.status()[0] == fails
    check(out, ref, noisy, label=case, alt=alt)


@pytest.mark.parametrize("recon", [WENOZ, VL, MP5, PPM, PPMX])
def test_flux_parity_further_reconstructions(recon):
    torch, gr = _setup()
    grid, P, _ = fm_torus(16, 16, 8)
    c = oracle.cfg(grid, gam=13 / 9, recon=recon)
    F_ref = oracle.fluxes(c, P, ct=True)
    s = gr.Grmhd(grid, 13 / 9, recon=recon)
    F = s.fluxes(torch.from_numpy(P)).cpu().numpy()
    n1, n2, n3 = grid.n1, grid.n2, grid.n3
    sl = [np.s_[:, 3:3 + n3, 3:3 + n2, 3:4 + n1], np.s_[:, 3:3 + n3, 3:4 + n2, 3:3 + n1],
          np.s_[:, 3:4 + n3, 3:3 + n2, 3:3 + n1]]
    for d in range(3):
        a, b = F[d][sl[d]], F_ref[d][sl[d]]
        scale = np.abs(b).max(axis=(1, 2, 3)) + 1e-300
        err = np.abs(a - b).max(axis=(1, 2, 3)) / scale
        assert err.max() < 1e-12, (d, err)


@pytest.mark.parametrize("recon", [WENOZ, VL, MP5, PPM, PPMX])
def test_torus128_full_step_further_reconstructions(recon):
    """The benchmark torus (128^3) with each reconstruction: one device-side
    CFL step, every zone against the oracle."""
    torch, gr = _setup()
    gam = 13 / 9
    grid, P, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    s = gr.Grmhd(grid, gam, recon=recon)
    s.load(torch.from_numpy(P).cuda())
    s.step_cfl()
    dt = s.last_dt()
    out = s.prims().cpu().numpy()
    c = oracle.cfg(grid, gam=gam, recon=recon, nthreads=THREADS)
    assert dt == pytest.approx(oracle.estimate_dt(c, P), rel=1e-14)
    ref, fails, _ = oracle.run(c, P, dt, 1)
    print("128^3 recon", recon, "failures", fails)
    check(out, ref, label="128^3 recon %d" % recon)
    assert s.status()[0] == fails


@pytest.mark.parametrize("recon", [WENOZ, VL, MP5, PPM, PPMX])
def test_mixed_precision_further_reconstructions(recon):
    """FP32 reconstruction and fluxes against the FP64 GPU path of the same
    reconstruction (3 steps of a 32 x 32 x 16 torus): density within 1e-4
    relative L1, div B at FP64 roundoff."""
    torch, gr = _setup()
    grid, P, _ = fm_torus(32, 32, 16)
    s64 = gr.Grmhd(grid, 13 / 9, recon=recon)
    s32 = gr.Grmhd(grid, 13 / 9, recon=recon, precision=gr.PREC_MIXED)
    s64.load(torch.from_numpy(P))
    s32.load(torch.from_numpy(P))
    dt = s64.dt()
    for _ in range(3):
        s64.step(dt)
        s32.step(dt)
    a, b = s32.prims().cpu().numpy(), s64.prims().cpu().numpy()
    r = rel_l1(a, b)
    print("mixed vs fp64 rel L1 per var", r)
    assert np.isfinite(a).all()
    assert r[0] < 1e-4
    mx, _ = s32.divb()
    scale = np.abs(interior(P[5:7])).max() / grid.dx[0]
    assert mx < 1e-13 * scale


def test_packs_and_adjoint_take_mc_or_weno5_only():
    torch, gr = _setup()
    g, blocks, _ = torus_pack(nblocks=4, n_global=32, sizes=(8,), probs=(1.0,), seed=4)
    for recon in (WENOZ, VL, MP5, PPM, PPMX):
        with pytest.raises(gr.GrmhdError):
            gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], 13 / 9, recon=recon)
