"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the host.

1. The library's primitive-variable recoveries -- 1D_W, Kastaun and the
   implicit solver's Newton-Raphson with its LDS-layout Jacobian -- and its
   zone-centre metric, compiled from the same source files as the GPU
   kernels (tests/host/inversion_host.cpp, with a stand-in for the HIP
   header), once with AddressSanitizer and UndefinedBehaviorSanitizer and
   once with MemorySanitizer (clang; an uninitialised read anywhere, the
   Jacobian's storage being fresh and uninitialised for every zone), on
   every zone of a torus: conserved variables of the torus with
   guesses 3 % off, and conserved variables of the state one oracle step
   later with the step's starting state as the guess (a stage inversion).
   Any out-of-range access, uninitialised use or undefined operation aborts
   the run; the recovered prims must also match the oracle's recovery of the
   same input (failure flags equal, prims to 1e-10 of the zone's scale plus
   the implicit solver's own stopping resolution, 1e-12 of max(|x|, 1e-3)
   for velocities, with a factor 10).
2. The library's geometric source of the momentum equations,
   (sqrt(-g)/2) T^{kl} d_nu g_kl for nu = 1, 2 from its metric-derivative
   rows (tests/host/source_host.cpp), against the oracle's connection form
   sqrt(-g) T^k_l Gamma^l_{nu k} on fuzzed Kerr states; the oracle's energy
   and x3-momentum sources, zero in a stationary axisymmetric metric, must
   come out zero to roundoff.
3. The adjoint's closed-form WENO5 gradient (tests/host/weno_grad_host.cpp)
   against the exact derivative of the same rational function (Python
   fractions) and against the dual-number WENO5; and its reverse-mode face
   state and zone terms (tests/host/face_vjp_host.cpp, zone_vjp_host.cpp)
   against dual-number evaluations of the same quantities, one seeded prim
   or the adiabatic index at a time.
4. The oracle itself (tests/host/oracle_driver.cpp), serially: SSPRK2 steps
   with each recovery, floors and the first-order flux correction,
   face-centred CT, Extended GRMHD, the CFL step and div B.  Results must
   equal the regular (OpenMP) oracle build bit for bit.

A sanitizer report makes the program exit non-zero with the report on
stderr, which the assertion shows.
"""

import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
from workloads import fm_torus, interior, RECON_MC, RECON_WENO5

HERE = os.path.dirname(os.path.abspath(__file__))
HOST = os.path.join(HERE, "host")
COMMON = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wno-unknown-pragmas"]
FLAGS = COMMON + ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
MSAN_FLAGS = COMMON + ["-fsanitize=memory", "-fsanitize-memory-track-origins=2"]
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", MSAN_OPTIONS="halt_on_error=1")


@pytest.fixture(scope="module")
def programs(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("sanitized")
    out = {}
    for name, src in (("inversion", "inversion_host.cpp"), ("oracle", "oracle_driver.cpp"),
                      ("source", "source_host.cpp"), ("weno_grad", "weno_grad_host.cpp"),
                      ("face_vjp", "face_vjp_host.cpp"), ("zone_vjp", "zone_vjp_host.cpp")):
        exe = str(d / name)
        subprocess.run(["g++", *FLAGS, "-I", HOST, "-o", exe, os.path.join(HOST, src)], check=True,
                       capture_output=True, text=True)
        out[name] = exe
    # MemorySanitizer (uninitialised reads) needs clang and its runtime
    msan = str(d / "inversion_msan")
    r = subprocess.run([CLANG, *MSAN_FLAGS, "-I", HOST, "-o", msan, os.path.join(HOST, "inversion_host.cpp")],
                       capture_output=True, text=True) if os.path.exists(CLANG) else None
    out["inversion_msan"] = msan if r is not None and r.returncode == 0 else None
    out["dir"] = d
    return out


def _run(exe, d, payload, tag):
    inp, outp = str(d / (tag + ".in")), str(d / (tag + ".out"))
    with open(inp, "wb") as f:
        f.write(payload)
    r = subprocess.run([exe, inp, outp], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    for report in ("runtime error", "AddressSanitizer", "MemorySanitizer"):
        assert report not in r.stderr, r.stderr[-4000:]
    return open(outp, "rb").read()


def _inversion_cases(grid, P, U, G):
    """x1, x2, U[8], guess[8] per interior zone (k, j, i order)."""
    x1, x2, _ = grid.centers()
    Ui, Gi = interior(U), interior(G)
    n3, n2, n1 = Ui.shape[1:]
    X1 = np.broadcast_to(x1[3:-3][None, None, :], (n3, n2, n1))
    X2 = np.broadcast_to(x2[3:-3][None, :, None], (n3, n2, n1))
    cases = np.concatenate([X1.reshape(1, -1), X2.reshape(1, -1), Ui.reshape(8, -1), Gi.reshape(8, -1)])
    return np.ascontiguousarray(cases.T)


@pytest.mark.parametrize("sanitizer", ["asan_ubsan", "msan"])
@pytest.mark.parametrize("inverter", [oracle.INV_1DW, oracle.INV_KASTAUN, oracle.INV_IMPLICIT],
                         ids=["1dw", "kastaun", "implicit"])
@pytest.mark.parametrize("kind", ["perturbed_guess", "stage"])
def test_library_recoveries_under_sanitizers(programs, inverter, kind, sanitizer):
    exe = programs["inversion"] if sanitizer == "asan_ubsan" else programs["inversion_msan"]
    if exe is None:
        pytest.skip("no clang with the MemorySanitizer runtime")
    grid, P, _ = fm_torus(16, 24, 8)
    gam = 13 / 9
    c = oracle.cfg(grid, gam=gam, recon=RECON_WENO5, inverter=inverter)
    if kind == "perturbed_guess":
        rng = np.random.default_rng(11)
        U = oracle.prims_to_cons(c, P)
        G = P * (1 + 0.03 * rng.uniform(-1, 1, P.shape))
    else:
        P1, _, _ = oracle.run(c, P, -1, 1)
        U = oracle.prims_to_cons(c, P1)
        G = P
    cases = _inversion_cases(grid, P, U, G)
    n = cases.shape[0]
    hdr = struct.pack("4i5d", n, inverter, 1, c.newton_maxit, gam, c.newton_tol, 1.0 - 1.0 / c.kastaun_wmax ** 2,
                      grid.a, grid.hslope)
    raw = _run(exe, programs["dir"], hdr + cases.tobytes(), "inv_%d_%s_%s" % (inverter, kind, sanitizer))
    got = np.frombuffer(raw[:8 * 8 * n], dtype=np.float64).reshape(n, 8)
    flags = np.frombuffer(raw[8 * 8 * n:], dtype=np.int32)
    ref, nfail, rflags = oracle.cons_to_prims(c, U, G)
    rp = interior(ref).reshape(8, -1).T
    rf = interior(rflags).reshape(-1)
    assert np.array_equal(flags != 0, rf != 0), (int(flags.sum()), int((rf != 0).sum()))
    ok = flags == 0
    # the implicit solver stops when every step is within 1e-12 max(|x|, f),
    # f = 1e-3 for the velocity components: two converged answers of a
    # velocity at rest may differ by that much
    fl = [0.0, 0.0, 1e-3, 1e-3, 1e-3, 0.0, 0.0, 0.0]
    for v, group in enumerate([[0], [1], [2, 3, 4], [2, 3, 4], [2, 3, 4], [5, 6, 7], [5, 6, 7], [5, 6, 7]]):
        scale = np.abs(rp[:, group]).sum(axis=1)
        scale = scale + 1e-10 * scale.max()
        err = np.abs(got[ok, v] - rp[ok, v])
        bar = 1e-10 * scale[ok] + 1e-11 * np.maximum(np.abs(rp[ok, v]), fl[v])
        worst = np.argmax(err / bar) if err.size else 0
        assert (err <= bar).all(), (v, err[worst], bar[worst])


def _oracle_job(programs, job, c, P, extra, dt, nsteps, tag):
    cb = bytes(memoryview(c))
    Pf = np.ascontiguousarray(P, dtype=np.float64)
    Xf = np.ascontiguousarray(extra if extra is not None else np.zeros(0), dtype=np.float64)
    payload = (struct.pack("iid", job, nsteps, dt) + cb + struct.pack("q", Pf.size) + Pf.tobytes() +
               struct.pack("q", Xf.size) + Xf.tobytes())
    raw = _run(programs["oracle"], programs["dir"], payload, tag)
    fails = struct.unpack("q", raw[:8])[0]
    o = 8
    Po = np.frombuffer(raw[o:o + 8 * Pf.size], dtype=np.float64).reshape(Pf.shape)
    o += 8 * Pf.size
    Xo = np.frombuffer(raw[o:o + 8 * Xf.size], dtype=np.float64).reshape(Xf.shape)
    o += 8 * Xf.size
    tail = np.frombuffer(raw[o:], dtype=np.float64)
    return fails, Po, Xo, tail


@pytest.mark.parametrize("opts", [dict(recon=RECON_WENO5), dict(recon=RECON_MC, inverter=oracle.INV_KASTAUN),
                                  dict(recon=RECON_WENO5, inverter=oracle.INV_IMPLICIT),
                                  dict(recon=RECON_MC, floors=True, fofc=True)],
                         ids=["weno5_1dw", "mc_kastaun", "weno5_implicit", "mc_floors_fofc"])
def test_oracle_steps_under_sanitizers(programs, opts):
    grid, P, _ = fm_torus(12, 12, 4)
    c = oracle.cfg(grid, gam=13 / 9, **opts)
    fails, Po, _, dts = _oracle_job(programs, 0, c, P, None, -1.0, 2, "step")
    ref, rfails, rdts = oracle.run(c, P, -1, 2)
    assert fails == rfails and np.array_equal(dts, rdts)
    assert np.array_equal(Po, ref)


def test_oracle_face_ct_emhd_dt_divb_under_sanitizers(programs):
    grid, P, info = fm_torus(12, 12, 4)
    c = oracle.cfg(grid, gam=13 / 9, recon=RECON_WENO5, ct=2)
    fails, Po, Fo, dts = _oracle_job(programs, 1, c, P, info["faces"], -1.0, 2, "face")
    ref, Fref, rfails, rdts = oracle.run_face(c, P, info["faces"], -1, 2)
    assert fails == rfails and np.array_equal(Po, ref) and np.array_equal(Fo, Fref)
    ce = oracle.cfg(grid, gam=13 / 9, recon=RECON_MC, integrator=oracle.INTEG_PC, tau_r=0.5, chi_emhd=0.2,
                    nu_emhd=0.2)
    X = np.zeros((2,) + P.shape[1:])
    X[:, 3:-3, 3:-3, 3:-3] = 1e-3 * np.random.default_rng(2).standard_normal((2, 4, 12, 12))
    fails, Po, Xo, dts = _oracle_job(programs, 2, ce, P, X, -1.0, 2, "emhd")
    ref, Xref, rfails, rdts = oracle.run_emhd(ce, P, X, -1, 2)
    assert fails == rfails and np.array_equal(Po, ref) and np.array_equal(Xo, Xref)
    c0 = oracle.cfg(grid, gam=13 / 9)
    _, _, _, tail = _oracle_job(programs, 3, c0, P, None, 0.0, 0, "dt")
    assert tail[0] == oracle.estimate_dt(c0, P)
    mx, mean = oracle.divb(c0, P)
    assert tail[1] == mx and tail[2] == mean


@pytest.mark.parametrize("metric", ["kerr", "flat"])
def test_library_geometric_source_against_the_oracle(programs, metric):
    import math
    from test_oracle_pins import _random_prims
    from workloads import GridSpec
    from workloads.torus import torus_grid
    grid = torus_grid(8, 8, 1) if metric == "kerr" else GridSpec(4, 4, 4)
    gam = 13.0 / 9.0
    c = oracle.cfg(grid, gam=gam)
    rng = np.random.default_rng(4)
    n = 2000
    if metric == "kerr":
        x1, x2 = rng.uniform(math.log(1.05), math.log(1000.0), n), rng.uniform(0.02, 0.98, n)
    else:
        x1, x2 = rng.uniform(0.0, 1.0, n), rng.uniform(0.0, 1.0, n)
    P = _random_prims(rng, n, c, x1, x2)
    hdr = struct.pack("2i3d", n, int(metric == "kerr"), gam, grid.a, grid.hslope)
    raw = _run(programs["source"], programs["dir"], hdr + np.column_stack([x1, x2, P]).tobytes(),
               "source_" + metric)
    got = np.frombuffer(raw, dtype=np.float64).reshape(n, 2)
    ref = np.array([oracle.point_source(c, P[q], x1[q], x2[q]) for q in range(n)])
    if metric == "flat":
        assert not got.any() and not ref.any()
        return
    mag = np.abs(ref[:, 2:4]).sum(axis=1)
    assert (mag > 0).all()
    # the two forms differ only in rounding (measured worst 1e-13 of |S1| + |S2|)
    for v in range(2):
        assert (np.abs(got[:, v] - ref[:, 2 + v]) <= 1e-12 * mag).all(), v
    # the oracle's energy and x3-momentum sources cancel to roundoff (measured 5e-15)
    assert (ref[:, 0] == 0.0).all()
    assert (np.abs(ref[:, 1]) <= 1e-13 * mag).all() and (np.abs(ref[:, 4]) <= 1e-13 * mag).all()
    assert (ref[:, 5:] == 0.0).all()


def _weno5_grad_exact(x, eps):
    """d weno5 / d x_z of the Jiang-Shu WENO5 edge value, in exact rational
    arithmetic (quotient rule on the weights' numerator and denominator)."""
    from fractions import Fraction as Fr
    a, b, c, d, e = [Fr(v) for v in x]
    eps = Fr(eps)
    t = [a - 2 * b + c, b - 2 * c + d, c - 2 * d + e]
    u = [a - 4 * b + 3 * c, b - d, 3 * c - 4 * d + e]
    dt = [[1, -2, 1, 0, 0], [0, 1, -2, 1, 0], [0, 0, 1, -2, 1]]
    du = [[1, -4, 3, 0, 0], [0, 1, 0, -1, 0], [0, 0, 3, -4, 1]]
    s = [eps + Fr(13, 12) * t[k] ** 2 + Fr(1, 4) * u[k] ** 2 for k in range(3)]
    ds = [[Fr(13, 6) * t[k] * dt[k][z] + Fr(1, 2) * u[k] * du[k][z] for z in range(5)] for k in range(3)]
    dk = [Fr(1, 10), Fr(6, 10), Fr(3, 10)]
    w = [dk[k] / s[k] ** 2 for k in range(3)]
    dw = [[-2 * dk[k] / s[k] ** 3 * ds[k][z] for z in range(5)] for k in range(3)]
    p = [(2 * a - 7 * b + 11 * c) / 6, (-b + 5 * c + 2 * d) / 6, (2 * c + 5 * d - e) / 6]
    dp = [[Fr(2, 6), Fr(-7, 6), Fr(11, 6), 0, 0], [0, Fr(-1, 6), Fr(5, 6), Fr(2, 6), 0],
          [0, 0, Fr(2, 6), Fr(5, 6), Fr(-1, 6)]]
    N, W = sum(w[k] * p[k] for k in range(3)), sum(w)
    return [float((sum(dw[k][z] * p[k] + w[k] * dp[k][z] for k in range(3)) * W -
                   N * sum(dw[k][z] for k in range(3))) / W ** 2) for z in range(5)]


def test_adjoint_reconstruction_gradients_closed_form(programs):
    """Rough, smooth (quadratic), small-scale and step stencils: the WENO5 closed
    form within 1e-11 of the exact derivative (measured 2.3e-12) and 2e-11
    of the dual-number form, relative to the sum of |exact derivatives|; the
    gradient sums to 1 (the edge value shifts with a constant added to the
    stencil); the MC edge values' closed-form gradients equal the dual ones
    bit for bit.  Exact ties between MC's candidates are added on purpose
    (flat and symmetric stencils)."""
    rng = np.random.default_rng(7)
    m, eps = 100, 1e-26
    xs = np.linspace(-0.2, 0.2, 5)
    X = np.concatenate([
        rng.normal(size=(m, 5)),
        np.array([a + b * xs + c * xs ** 2 for a, b, c in rng.normal(size=(m, 3))]),
        10 ** rng.uniform(-6, 0, (m, 1)) * (1 + 0.01 * rng.normal(size=(m, 5))),
        np.where(rng.random((m, 5)) < 0.5, 1.0, 0.1) * rng.uniform(0.5, 2, (m, 1)) *
        (1 + 1e-3 * rng.normal(size=(m, 5)))])
    n = len(X)
    # MC's switching points: ties between |2 dl|, |2 dr|, |dc/2|, flat and sign changes
    T = np.array([[0, 1, 2, 3, 4], [1, 1, 1, 1, 1], [0, 1, 1, 2, 2], [0, 2, 3, 4, 6], [3, 1, 2, 0, 1],
                  [0, 0, 1, 1, 0], [1, 0, 0, 1, 1], [2, 1, 0, -1, -2]], dtype=np.float64)
    raw = _run(programs["weno_grad"], programs["dir"],
               struct.pack("<id", n + len(T), eps) + np.concatenate([X, T]).tobytes(), "weno_grad")
    extra = np.frombuffer(raw, dtype=np.float64).reshape(n + len(T), 22)[n:]
    assert np.array_equal(extra[:, 10:16], extra[:, 16:22])
    raw = raw[:n * 22 * 8]
    out = np.frombuffer(raw, dtype=np.float64).reshape(n, 22)
    closed, dual = out[:, :5], out[:, 5:10]
    # the MC edge values: piecewise linear, so the closed form is the dual
    # derivative bit for bit (all factors are powers of two)
    assert np.array_equal(out[:, 10:16], out[:, 16:22])
    exact = np.array([_weno5_grad_exact(x, eps) for x in X])
    scale = np.abs(exact).sum(axis=1)
    assert (np.abs(closed - exact).max(axis=1) <= 1e-11 * scale).all()
    assert (np.abs(closed - dual).max(axis=1) <= 2e-11 * scale).all()
    assert np.abs(closed.sum(axis=1) - 1.0).max() < 1e-13


@pytest.mark.parametrize("direction", [1, 2, 3])
def test_adjoint_reverse_mode_face_state(programs, direction):
    """Fuzzed Kerr states (rho, u, velocities and fields over several
    decades, adiabatic index in [1.1, 1.7]) with random adjoints of the
    state's flux, conserved variables and both speeds: the reverse sweep's
    adjoint of each prim and of the adiabatic index equals the dual-number
    directional products within 1e-10 of the sum of the products' terms
    (measured worst 1.1e-11 over the three directions, median 1e-16)."""
    import math
    from test_oracle_pins import _random_prims
    from workloads.torus import torus_grid
    grid = torus_grid(8, 8, 1)
    c = oracle.cfg(grid, gam=13.0 / 9.0)
    rng = np.random.default_rng(5 + direction)
    n = 1500
    x1, x2 = rng.uniform(math.log(1.05), math.log(1000.0), n), rng.uniform(0.02, 0.98, n)
    P = _random_prims(rng, n, c, x1, x2)
    rows = np.column_stack([x1, x2, rng.uniform(1.1, 1.7, n), P, rng.normal(size=(n, 18))])
    hdr = struct.pack("<3i2d", n, 1, direction, grid.a, grid.hslope)
    raw = _run(programs["face_vjp"], programs["dir"], hdr + rows.tobytes(), "face_vjp_%d" % direction)
    out = np.frombuffer(raw, dtype=np.float64).reshape(n, 27)
    rev, dual, scale = out[:, :9], out[:, 9:18], out[:, 18:]
    assert np.isfinite(rev).all()
    assert (np.abs(rev - dual) <= 1e-10 * scale).all()


@pytest.mark.parametrize("with_u", [False, True], ids=["source", "source_and_conserved"])
def test_adjoint_reverse_mode_zone_terms(programs, with_u):
    """The zone's geometric source through the connection (adjoints of its
    four components) and, for the first stage, its conserved variables:
    the reverse sweep equals the dual-number directional products within
    1e-9 of the sum of the products' terms (measured worst 5e-11 for the
    source alone, where the connection sums cancel; median 2e-16)."""
    import math
    from test_oracle_pins import _random_prims
    from workloads.torus import torus_grid
    grid = torus_grid(8, 8, 1)
    c = oracle.cfg(grid, gam=13.0 / 9.0)
    rng = np.random.default_rng(9 + int(with_u))
    n = 1500
    x1, x2 = rng.uniform(math.log(1.05), math.log(1000.0), n), rng.uniform(0.02, 0.98, n)
    P = _random_prims(rng, n, c, x1, x2)
    rows = np.column_stack([x1, x2, rng.uniform(1.1, 1.7, n), P, rng.normal(size=(n, 12))])
    hdr = struct.pack("<3i2d", n, 1, int(with_u), grid.a, grid.hslope)
    raw = _run(programs["zone_vjp"], programs["dir"], hdr + rows.tobytes(), "zone_vjp_%d" % int(with_u))
    out = np.frombuffer(raw, dtype=np.float64).reshape(n, 27)
    rev, dual, scale = out[:, :9], out[:, 9:18], out[:, 18:]
    assert np.isfinite(rev).all()
    assert (np.abs(rev - dual) <= 1e-9 * scale).all()
