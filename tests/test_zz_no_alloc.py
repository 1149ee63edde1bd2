"""The allocation-free CFL step (grmhd_cfl_dt_noalloc) against the context's
grmhd_estimate_dt on the same prims: two calls in a row on one GPU, the
second on a smaller grid (the shared scratch keeps the first call's
contents), each equal bit for bit, and a NaN zone reported as E_STATE."""

import numpy as np
import pytest

from workloads import fm_torus, linear_mode, RECON_WENO5, RECON_MC

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01361_amd import grmhd as gr
    return torch, gr


def test_noalloc_cfl_step_matches_the_context_entry_point():
    torch, gr = _setup()
    cases = [(fm_torus(48, 40, 24)[0:2], 13 / 9, RECON_WENO5),
             (fm_torus(16, 12, 4)[0:2], 13 / 9, RECON_MC),
             (linear_mode("fast", 24, ndim=3)[0:2], 4 / 3, RECON_MC)]
    for (grid, P), gam, recon in cases:
        print("grid", grid.n1, grid.n2, grid.n3, flush=True)
        Pt = torch.from_numpy(P).cuda()
        s = gr.Grmhd(grid, gam, recon=recon)
        s.load(Pt)
        expect = s.dt()
        got = gr.cfl_dt_noalloc(grid, gam, Pt, recon=recon)
        print("context", expect, "no-alloc", got, flush=True)
        assert got == expect
        s.close()


def test_noalloc_cfl_step_flags_a_nan_zone():
    torch, gr = _setup()
    grid, P, _ = fm_torus(16, 12, 4)
    P = P.copy()
    P[0, 5, 6, 7] = np.nan
    with pytest.raises(gr.GrmhdError, match="-3"):
        gr.cfl_dt_noalloc(grid, 13 / 9, torch.from_numpy(P).cuda())
