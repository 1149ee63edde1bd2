"""Uneven packs of torus meshblocks.

torus_pack: each block is a seeded sub-box [i0, i0+n) x [j0, j0+n) x
[k0, k0+n) of the n_global^3 torus grid, n drawn from `sizes` with
probabilities `probs`, the offsets uniform in [0, n_global - n].  Its ghost
zones hold the global initial data (frozen, Dirichlet), so every block is an
independent domain whose coordinates are the matching sub-range of the
global grid.

torus_tiling: blocks that tile the whole grid once, as an octree would: the
grid is cut into blocks of the largest size, and each block is split into
eight of half its size with probability `split` (seeded), recursively down to
the smallest size.  Ghost zones start from the global padded initial data;
with the pack's ghost exchange on, the tiling advances as the global grid.
"""

import numpy as np

from .spec import GridSpec, NG, BC_FROZEN
from .torus import fm_torus


def torus_pack(nblocks=320, n_global=128, sizes=(16, 32, 64),
               probs=(0.6, 0.3, 0.1), seed=7, torus_seed=1, gamma=13.0 / 9.0):
    g, P, info = fm_torus(n_global, n_global, n_global, seed=torus_seed,
                          gamma=gamma)
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=nblocks, p=np.asarray(probs))
    d1, d2, d3 = g.dx
    blocks = []
    for n in ns:
        n = int(n)
        i0, j0, k0 = (int(v) for v in rng.integers(0, n_global - n + 1, size=3))
        sub = np.ascontiguousarray(
            P[:, k0:k0 + n + 2 * NG, j0:j0 + n + 2 * NG, i0:i0 + n + 2 * NG])
        bg = GridSpec(n, n, n,
                      x1min=g.x1min + i0 * d1, x1max=g.x1min + (i0 + n) * d1,
                      x2min=g.x2min + j0 * d2, x2max=g.x2min + (j0 + n) * d2,
                      x3min=g.x3min + k0 * d3, x3max=g.x3min + (k0 + n) * d3,
                      bc=(BC_FROZEN,) * 6, metric=g.metric, a=g.a,
                      hslope=g.hslope)
        blocks.append(dict(n=n, offset=(i0, j0, k0), grid=bg, prims=sub))
    return g, blocks, info


def _block(g, P, n, i0, j0, k0):
    d1, d2, d3 = g.dx
    sub = np.ascontiguousarray(P[:, k0:k0 + n + 2 * NG, j0:j0 + n + 2 * NG, i0:i0 + n + 2 * NG])
    bg = GridSpec(n, n, n,
                  x1min=g.x1min + i0 * d1, x1max=g.x1min + (i0 + n) * d1,
                  x2min=g.x2min + j0 * d2, x2max=g.x2min + (j0 + n) * d2,
                  x3min=g.x3min + k0 * d3, x3max=g.x3min + (k0 + n) * d3,
                  bc=(BC_FROZEN,) * 6, metric=g.metric, a=g.a, hslope=g.hslope)
    return dict(n=n, offset=(i0, j0, k0), grid=bg, prims=sub)


def tiling(g, P, sizes=(16, 32), split=0.5, seed=3):
    """Octree-like uneven tiling of the cubic grid g (padded prims P) by
    blocks of the given sizes (each a power-of-two multiple of the next)."""
    sizes = sorted(int(s) for s in sizes)
    top = sizes[-1]
    n_global = g.n1
    assert g.n2 == n_global and g.n3 == n_global
    assert n_global % top == 0 and all(top % s == 0 for s in sizes)
    rng = np.random.default_rng(seed)
    blocks = []

    def place(n, i0, j0, k0):
        smaller = [s for s in sizes if s < n]
        if smaller and rng.random() < split:
            h = n // 2 if (n // 2) in sizes else smaller[-1]
            for dk in range(0, n, h):
                for dj in range(0, n, h):
                    for di in range(0, n, h):
                        place(h, i0 + di, j0 + dj, k0 + dk)
        else:
            blocks.append(_block(g, P, n, i0, j0, k0))

    for k0 in range(0, n_global, top):
        for j0 in range(0, n_global, top):
            for i0 in range(0, n_global, top):
                place(top, i0, j0, k0)
    return blocks


def torus_tiling(n_global=64, sizes=(16, 32), split=0.5, seed=3, torus_seed=1,
                 gamma=13.0 / 9.0, magnetised=True):
    g, P, info = fm_torus(n_global, n_global, n_global, seed=torus_seed, gamma=gamma,
                          magnetised=magnetised)
    return g, tiling(g, P, sizes, split, seed), P, info
