"""Batched uneven packs: three launches per stage (fluxes, EMFs, update) over many blocks.

Every block of a pack must match the same block advanced alone through the
single-block path bit for bit, and the pack as a whole the FP64 oracle
(frozen ghosts, block by block) to the parity bar; tile shapes change nothing
in the results.  With the ghost exchange on, blocks that tile a grid must
advance as that grid: against the single GPU grid and the oracle's global
run to the parity bar (torus), bit for bit where the block spacings equal
the grid's exactly (flat periodic fast mode).
"""

import numpy as np
import pytest

import oracle
from parity_util import GROUPS, ZONE_TOL
from parity_util import rel_l1, zone_rel
from workloads import (torus_pack, torus_tiling, tiling, linear_mode, interior, RECON_MC, RECON_WENO5,
                       NG)

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01361_amd import grmhd as gr
    return torch, gr


def _packed(blocks):
    return np.concatenate([b["prims"].ravel() for b in blocks])


def _unpack(flat, blocks):
    out, o = [], 0
    for b in blocks:
        n = b["n"] + 6
        out.append(flat[o:o + 8 * n ** 3].reshape(8, n, n, n))
        o += 8 * n ** 3
    return out


@pytest.mark.parametrize("recon,inv", [(RECON_MC, 0), (RECON_WENO5, 0), (RECON_MC, 1)],
                         ids=["mc", "weno5", "mc_kastaun"])
def test_pack_matches_single_blocks_and_oracle(recon, inv):
    torch, gr = _setup()
    g, blocks, _ = torus_pack(nblocks=12, n_global=32, sizes=(8, 16), probs=(0.5, 0.5), seed=4)
    gam = 13 / 9
    single = gr.Grmhd(g, gam, recon=recon)
    from workloads import fm_torus
    _, Pg, _ = fm_torus(32, 32, 32)
    single.load(torch.from_numpy(Pg).cuda())
    dt = single.dt()
    pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], gam, recon=recon,
                 inverter=inv)
    pk.load(torch.from_numpy(_packed(blocks)).cuda())
    for _ in range(2):
        pk.step(dt)
    res = _unpack(pk.prims().cpu().numpy(), blocks)
    num = np.zeros(8)
    den = np.zeros(8)
    zone = np.zeros(8)
    for b, out in zip(blocks, res):
        s = gr.Grmhd(b["grid"], gam, recon=recon, inverter=inv)
        s.load(torch.from_numpy(b["prims"]).cuda())
        for _ in range(2):
            s.step(dt)
        alone = s.prims().cpu().numpy()
        assert np.array_equal(interior(out), interior(alone)), b["offset"]
        c = oracle.cfg(b["grid"], gam=gam, recon=recon, inverter=inv)
        ref, _, _ = oracle.run(c, b["prims"], dt, 2)
        zone = np.maximum(zone, zone_rel(out, ref))
        # the pack is one workload: its relative L1 sums over all blocks
        A, B = interior(out), interior(ref)
        for v in range(8):
            num[v] += np.abs(A[v] - B[v]).sum()
            den[v] += sum(np.abs(B[w]).sum() for w in GROUPS[v])
    rel = num / den
    print("pack vs oracle rel L1", rel, "per zone", zone)
    assert rel.max() <= 1e-12, rel
    assert np.all(zone <= ZONE_TOL), zone


def test_pack_tile_shapes_do_not_change_results():
    torch, gr = _setup()
    g, blocks, _ = torus_pack(nblocks=10, n_global=32, sizes=(8, 16), probs=(0.5, 0.5), seed=6)
    gam = 13 / 9
    flat = torch.from_numpy(_packed(blocks)).cuda()
    outs = []
    for tiles in ({8: (0, 0, 0), 16: (0, 0, 0)}, {8: (8, 8, 4), 16: (16, 16, 1)},
                  {8: (4, 8, 8), 16: (16, 4, 4)}, {8: (8, 4, 2), 16: (32, 2, 2)}):
        pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], gam, recon=RECON_WENO5)
        for n, t in tiles.items():
            pk.set_tiles(n, *t)
        pk.load(flat)
        pk.step(1e-3)
        outs.append(pk.prims().cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def _tiled_interior(flat, blocks, shape):
    """The global interior assembled from a tiling's blocks."""
    out = np.zeros((8,) + shape)
    for b, q in zip(blocks, _unpack(flat, blocks)):
        i, j, k = b["offset"]
        n = b["n"]
        out[:, k:k + n, j:j + n, i:i + n] = interior(q)
    return out


@pytest.mark.parametrize("recon", [RECON_MC, RECON_WENO5])
def test_tiling_with_ghost_exchange_advances_as_the_global_grid(recon):
    """An uneven octree-like tiling of the 64^3 torus (48 blocks of 16^3 and
    2 of 32^3) with the ghost exchange on: two steps match the single global
    grid on the GPU and the oracle's global run to the parity bar, with the
    same failure count; with frozen ghosts the blocks drift apart from it."""
    torch, gr = _setup()
    gam = 13 / 9
    g, blocks, P, _ = torus_tiling(64, sizes=(16, 32), split=0.5, seed=3, gamma=gam)
    print("tiling", len(blocks), "blocks, recon", recon, flush=True)
    single = gr.Grmhd(g, gam, recon=recon)
    single.load(torch.from_numpy(P).cuda())
    dt = single.dt()
    for _ in range(2):
        single.step(dt)
    ref_gpu = interior(single.prims().cpu().numpy())
    ref, fails, _ = oracle.run(oracle.cfg(g, gam=gam, recon=recon), P, dt, 2)
    pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], gam, recon=recon)
    pk.set_exchange(True)
    pk.load(torch.from_numpy(_packed(blocks)).cuda())
    for _ in range(2):
        pk.step(dt)
    shape = (64, 64, 64)
    out = _tiled_interior(pk.prims().cpu().numpy(), blocks, shape)
    pad = lambda A: np.pad(A, ((0, 0), (NG, NG), (NG, NG), (NG, NG)))
    r_gpu = rel_l1(pad(out), pad(ref_gpu))
    r_orc = rel_l1(pad(out), ref)
    print("tiling vs single grid", r_gpu, "vs oracle", r_orc, "fails", pk.status(), single.status()[0], fails)
    assert r_gpu.max() <= 1e-12 and r_orc.max() <= 1e-12
    z = zone_rel(pad(out), ref)
    assert np.all(z <= ZONE_TOL), z
    assert pk.status() == single.status()[0] == fails
    # frozen ghosts: the same tiling no longer advances as the global grid
    pk.set_exchange(False)
    pk.load(torch.from_numpy(_packed(blocks)).cuda())
    for _ in range(2):
        pk.step(dt)
    frozen = _tiled_interior(pk.prims().cpu().numpy(), blocks, shape)
    assert rel_l1(pad(frozen), pad(ref_gpu)).max() > 1e-9


@pytest.mark.parametrize("recon", [RECON_MC, RECON_WENO5])
def test_periodic_tiling_with_exchange_is_the_global_grid_bit_for_bit(recon):
    """The 3-D fast mode (flat, periodic, 32^3) tiled by blocks of 8 and 16
    with the exchange on: the block spacings equal the grid's exactly and
    the metric is constant, so three steps reproduce the single grid bit for
    bit, wraps across every periodic face included."""
    torch, gr = _setup()
    g, P, _, _ = linear_mode("fast", 32, ndim=3)
    blocks = tiling(g, P, sizes=(8, 16), split=0.5, seed=2)
    print("periodic tiling", len(blocks), "blocks", flush=True)
    single = gr.Grmhd(g, 4 / 3, recon=recon)
    single.load(torch.from_numpy(P).cuda())
    dt = single.dt()
    pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], 4 / 3, recon=recon)
    pk.set_exchange(True)
    pk.load(torch.from_numpy(_packed(blocks)).cuda())
    for _ in range(3):
        single.step(dt)
        pk.step(dt)
    out = _tiled_interior(pk.prims().cpu().numpy(), blocks, (32, 32, 32))
    assert np.array_equal(out, interior(single.prims().cpu().numpy()))


def test_ghost_exchange_rejects_overlapping_blocks():
    torch, gr = _setup()
    g, blocks, _ = torus_pack(nblocks=4, n_global=32, sizes=(16,), probs=(1.0,), seed=4)
    pk = gr.Pack(g, [16, 16], [(0, 0, 0), (8, 0, 0)], 13 / 9, recon=RECON_MC)
    with pytest.raises(gr.GrmhdError):
        pk.set_exchange(True)
