"""Pins of the seeded initial data against closed forms."""

import math

import numpy as np
import pytest

from workloads import linear_mode, fm_torus, torus_pack, torus_tiling, interior, NG
from workloads.linear_modes import select_mode
from workloads.torus import fm_ell, fm_lnh, _mks_metric, _bsq


def test_mode_speeds_match_rest_frame_dispersion_relation():
    """Phase speeds are the roots of
    v^4 - [vA^2 + cs^2 (1 - vA^2 cos^2) ... ] v^2 + cs^2 vA^2 cos^2 = 0."""
    gam, rho, u = 4 / 3, 1.0, 1.0
    p = (gam - 1) * u
    w = rho + u + p
    cs2 = gam * p / w
    va2 = 1.0 / (1.0 + w)              # |B| = 1
    cos2 = 0.5                         # k along (1,1,0), B along x
    b = va2 + cs2 * (1 - va2) + cs2 * va2 * cos2
    c = cs2 * va2 * cos2
    fast = math.sqrt((b + math.sqrt(b * b - 4 * c)) / 2)
    slow = math.sqrt((b - math.sqrt(b * b - 4 * c)) / 2)
    assert select_mode("fast")[0] == pytest.approx(fast, rel=1e-13)
    assert select_mode("slow")[0] == pytest.approx(slow, rel=1e-13)
    assert select_mode("alfven")[0] == pytest.approx(math.sqrt(va2 * cos2), rel=1e-13)


def test_mode_perturbations_are_divergence_free_and_normalised():
    for name in ("fast", "slow", "alfven"):
        s, r = select_mode(name)
        assert np.linalg.norm(r) == pytest.approx(1.0)
        assert abs(r[5] + r[6]) < 1e-14          # k . dB = 0 for k = (1, 1, 0)


def test_fm_torus_constants():
    a, rmax, rin = 0.9375, 12.0, 6.0
    ell = fm_ell(a, rmax)
    assert ell == pytest.approx(4.281284468531897, rel=1e-14)
    r = np.linspace(rin, 40.0, 340001)
    lnh = fm_lnh(r, np.full_like(r, np.pi / 2), a, ell, rin)
    assert abs(lnh[0]) < 1e-14
    assert r[np.argmax(lnh)] == pytest.approx(rmax, abs=2e-4)


def test_fm_torus_state():
    n = 32
    g, P, info = fm_torus(n, n, 4)
    assert np.isfinite(P).all()
    I = interior(P)
    assert I[0].max() == pytest.approx(1.0, rel=0.05)        # perturbation is on u only
    x1, x2, _ = g.centers()
    X2, X1 = np.meshgrid(x2, x1, indexing="ij")
    gcov, gdet, gtt, gt1 = _mks_metric(X1, X2, g.a, g.hslope)
    # minimum plasma beta over magnetised zones equals 100
    gc = np.broadcast_to(gcov[:, :, None], (4, 4) + P.shape[1:])
    bsq = _bsq(P, gc, gtt[None], gt1[None])
    bi = interior(bsq)
    m = bi > 0
    beta = 2 * (13 / 9 - 1) * interior(P[1])[m] / bi[m]
    assert beta.min() == pytest.approx(100.0, rel=1e-12)


def test_pack_is_seeded_and_uses_global_data():
    g, blocks, _ = torus_pack(nblocks=12, n_global=32, sizes=(8, 16), probs=(0.5, 0.5), seed=3)
    g2, blocks2, _ = torus_pack(nblocks=12, n_global=32, sizes=(8, 16), probs=(0.5, 0.5), seed=3)
    _, P, _ = fm_torus(32, 32, 32)
    for b, b2 in zip(blocks, blocks2):
        assert b["offset"] == b2["offset"] and np.array_equal(b["prims"], b2["prims"])
        i0, j0, k0 = b["offset"]
        n = b["n"]
        assert np.array_equal(b["prims"], P[:, k0:k0 + n + 2 * NG, j0:j0 + n + 2 * NG, i0:i0 + n + 2 * NG])


def test_tiling_covers_the_grid_once_with_the_global_data():
    """The uneven octree-like tiling covers every zone of the grid exactly
    once, uses every requested size, and each block's padded prims are the
    global padded prims over its sub-box."""
    g, blocks, P, _ = torus_tiling(64, sizes=(16, 32), split=0.5, seed=3)
    cover = np.zeros((64, 64, 64), int)
    for b in blocks:
        i, j, k = b["offset"]
        n = b["n"]
        cover[k:k + n, j:j + n, i:i + n] += 1
        assert np.array_equal(b["prims"], P[:, k:k + n + 2 * NG, j:j + n + 2 * NG, i:i + n + 2 * NG])
        assert b["grid"].x1min == pytest.approx(g.x1min + i * g.dx[0], rel=1e-15, abs=1e-15)
    assert cover.min() == 1 and cover.max() == 1
    assert {b["n"] for b in blocks} == {16, 32}
    _, again, _, _ = torus_tiling(64, sizes=(16, 32), split=0.5, seed=3)
    assert [b["offset"] for b in again] == [b["offset"] for b in blocks]


def test_michel_solution_constants_and_sonic_point():
    """The Michel flow: mass flux and Bernoulli constant are the same at every
    zone centre, the flow is supersonic inside the sonic radius and subsonic
    outside, and at r_c the sound speed and u^r meet Michel's conditions."""
    import math
    from workloads import bondi, michel_constants, michel_rho
    g, P, c = bondi(48, 4)
    x1, _, _ = g.centers()
    r = np.exp(x1)
    rho = P[0, 3, 3]
    gam = c["gamma"]
    theta = c["K"] * rho ** (gam - 1.0)
    h = 1.0 + gam / (gam - 1.0) * theta
    ur = -c["mdot"] / (4.0 * math.pi * r * r * rho)
    bern = h * h * (1.0 - 2.0 / r + ur * ur)
    assert np.allclose(bern, c["bern"], rtol=1e-12)
    cs2 = gam * theta / h
    # the radial velocity measured by a static observer exceeds the sound
    # speed exactly inside r_c
    outside = r > 2.0
    v2 = ur[outside] ** 2 / (1.0 - 2.0 / r[outside] + ur[outside] ** 2)
    assert np.all((v2 > cs2[outside]) == (r[outside] < c["rc"]))
    rc = c["rc"]
    rho_c = michel_rho(rc, c)
    th_c = c["K"] * rho_c ** (gam - 1.0)
    urc = c["mdot"] / (4.0 * math.pi * rc * rc * rho_c)
    assert urc ** 2 == pytest.approx(1.0 / (2.0 * rc), rel=1e-8)
    cs2c = gam * th_c / (1.0 + gam / (gam - 1.0) * th_c)
    assert cs2c == pytest.approx(urc ** 2 / (1.0 - 3.0 * urc ** 2), rel=1e-8)
    c2 = michel_constants(rc=rc, gamma=gam, rho_c=2.0)
    assert c2["K"] * 2.0 ** (gam - 1.0) == pytest.approx(c["K"], rel=1e-14)


def test_magnetised_blast_set_up():
    from workloads import magnetised_blast, interior
    grid, P = magnetised_blast(48)
    I = interior(P)
    assert P.shape == (8, 7, 54, 54)
    rho, u = I[0], I[1]
    assert rho.max() == pytest.approx(1e-2) and rho.min() == pytest.approx(1e-4)
    p = u / 3.0                                        # gamma = 4/3
    assert p.max() == pytest.approx(1.0) and p.min() == pytest.approx(3e-5)
    assert np.all(I[2:5] == 0) and np.all(I[5] == 0.07) and np.all(I[6:] == 0)
    # b^2/rho = 49 in the ambient gas, at rest
    assert (0.07 ** 2 / rho.min()) == pytest.approx(49.0)
    # symmetric under x -> -x and y -> -y
    assert np.array_equal(I[0], I[0][:, ::-1, :]) and np.array_equal(I[0], I[0][:, :, ::-1])


def test_face_fields_of_the_workloads():
    """Face fields for face-centred CT: zero face divergence, and (torus)
    their zone means over sqrt(-g) are the zone-centred B of the prims."""
    import oracle
    from workloads import magnetised_blast, linear_mode_faces, torus_grid
    grid, P, info = fm_torus(24, 24, 8)
    F = info["faces"]
    c = oracle.cfg(grid, gam=13 / 9, ct=2)
    mx, _ = oracle.face_divb(c, F)
    assert mx < 1e-14 * np.abs(F).max() / min(grid.dx)
    P0 = oracle.run_face(c, P, F, 1e-30, 0)[0]
    I0, I = interior(P0), interior(P)
    assert np.abs(I0[5:7] - I[5:7]).max() < 1e-12 * np.abs(I[5:7]).max()
    g, P, F, _, _ = linear_mode_faces("fast", 16, ndim=3)
    mx, _ = oracle.face_divb(oracle.cfg(g, ct=2), F)
    assert mx < 1e-12
    g, P, F = magnetised_blast(24, faces=True)
    assert np.all(F[0] == 0.07) and np.all(F[1:] == 0)
