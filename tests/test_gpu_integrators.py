"""GPU-vs-oracle parity of the other time integrators: predictor-corrector,
RK1 (forward Euler) and SSPRK(5,4), through the C ABI.

Bars as for SSPRK2 (parity_util.check): relative L1 per primitive at most
1e-12 per step, every zone within the per-zone bars, failure counts equal,
the u~ of a linear mode at rest held to 3x the oracle's own FMA spread on
the case.  RK1's one stage (SSPRK(5,4)'s fifth)
writes the CFL-rate partials itself, so a device-side CFL step must equal
a host-dt step with the dt the oracle estimates.
"""

import numpy as np
import pytest

import oracle
from parity_util import rel_l1, check, NOISY_MODE
from workloads import linear_mode, fm_torus, bondi, interior, RECON_MC, RECON_WENO5

pytestmark = pytest.mark.gpu

TOL = 1e-12
PC, RK1, SSP54 = oracle.INTEG_PC, oracle.INTEG_RK1, oracle.INTEG_SSPRK54


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01361_amd import grmhd as gr
    return torch, gr


CASES = {
    "fast32_mc": lambda: (linear_mode("fast", 32, ndim=3)[0:2], 4 / 3, RECON_MC, NOISY_MODE),
    "torus24_weno": lambda: (fm_torus(24, 24, 8)[0:2], 13 / 9, RECON_WENO5, ()),
    "torus20x28x6_mc": lambda: (fm_torus(20, 28, 6)[0:2], 13 / 9, RECON_MC, ()),
    "bondi32x16_mc": lambda: (bondi(32, 16)[0:2], 4 / 3, RECON_MC, ()),
}


@pytest.mark.parametrize("integ", [PC, RK1, SSP54], ids=["pc", "rk1", "ssprk54"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_step_parity_integrators(case, integ):
    torch, gr = _setup()
    (grid, P), gam, recon, noisy = CASES[case]()
    print("case", case, "integrator", integ, flush=True)
    c = oracle.cfg(grid, gam=gam, recon=recon, integrator=integ)
    ref, fails, dts, _ = oracle.run(c, P, -1, 3, flags=True)
    alt = oracle.run(c, P, -1, 3, fma=True)[0] if noisy else None
    s = gr.Grmhd(grid, gam, recon=recon, integrator=integ)
    s.load(torch.from_numpy(P))
    for dt in dts:
        s.step(dt)
    out = s.prims().cpu().numpy()
    print(case, integ, "fails", fails, s.status()[0], )
    assert s.status()[0] == fails
    check(out, ref, noisy, label="%s %d" % (case, integ), alt=alt)


@pytest.mark.parametrize("integ", [PC, RK1, SSP54], ids=["pc", "rk1", "ssprk54"])
def test_device_cfl_step_integrators(integ):
    """Device-side CFL steps: each step's dt is the oracle's CFL estimate of
    the state it starts from (the partials the previous step's last stage
    wrote -- RK1's only stage, PC's corrector, SSPRK(5,4)'s fifth stage),
    and the steps match the oracle run at those dts."""
    torch, gr = _setup()
    grid, P, _ = fm_torus(24, 24, 8)
    c = oracle.cfg(grid, gam=13 / 9, recon=RECON_WENO5, integrator=integ)
    s = gr.Grmhd(grid, 13 / 9, recon=RECON_WENO5, integrator=integ)
    s.load(torch.from_numpy(P))
    got = []
    for _ in range(3):
        expect = oracle.estimate_dt(c, s.prims().cpu().numpy())
        s.step_cfl()
        got.append(s.last_dt())
        assert got[-1] == pytest.approx(expect, rel=1e-14)
    ref = P
    for dt in got:
        ref, _, _ = oracle.run(c, ref, dt, 1)
    check(s.prims().cpu().numpy(), ref, label="device CFL %d" % integ)


def test_torus128_integrators_full_step():
    """The benchmark torus (128^3, WENO5): one device-side CFL step with
    each integrator, every zone against the oracle."""
    torch, gr = _setup()
    import os
    gam = 13 / 9
    grid, P, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    for integ in (PC, RK1, SSP54):
        s = gr.Grmhd(grid, gam, recon=RECON_WENO5, integrator=integ)
        s.load(torch.from_numpy(P).cuda())
        s.step_cfl()
        dt = s.last_dt()
        out = s.prims().cpu().numpy()
        c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, integrator=integ,
                       nthreads=min(16, os.cpu_count() or 1))
        ref, fails, _ = oracle.run(c, P, dt, 1)
        print("128^3 integrator", integ, "failures", fails)
        check(out, ref, label="128^3 integrator %d" % integ)
        assert s.status()[0] == fails
        del s


def test_other_integrators_take_the_plain_path_only():
    torch, gr = _setup()
    grid, P, _ = fm_torus(16, 16, 4)
    for integ in (gr.INTEG_PC, gr.INTEG_RK1, gr.INTEG_SSPRK54):
        for kw in (dict(floors=True), dict(fofc=True), dict(ct=gr.CT_FACE_AVG), dict(inverter=gr.INV_IMPLICIT)):
            with pytest.raises(gr.GrmhdError):
                gr.Grmhd(grid, 13 / 9, integrator=integ, **kw)
