"""Throughput of the HARM ideal-GRMHD step on one MI355X.

Headline workload: the magnetised Fishbone-Moncrief torus in Kerr a = 0.9375,
modified Kerr-Schild coordinates (h = 0.3, r from 0.95 r+ to 1000), r_in = 6,
r_max = 12, gamma = 13/9, beta_min = 100, u perturbed by +-4 % (seed 1),
128^3 zones, WENO5, FP64.  A step is one SSPRK2 step -- both stages: ghost
fill, reconstruction + face states + LLF fluxes along x1..x3, Flux-CT EMFs,
divergence + source + RK combination + 1D_W inversion -- plus the CFL dt
reduction that chooses it.  Inputs are resident in HBM before timing starts.

One JSON line: zone-cycles per second, the roofline of the dominant kernel
(its duration from HIP events recorded on the library's stream over the timed
region), the FP64 CPU oracle timed on a bounded sample, and the reduced-
precision and batched forms measured against plain FP64 on the same GPU.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks.
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# Algorithmic work per unit (a flux unit is one face, an update unit one
# zone), flops from the oracle's counting build (every +, -, *, /, sqrt is
# one flop; python -m oracle.count_flops), bytes that must cross HBM once:
#   flux:   read 8 prims + write 8 flux components           = 128 B per face
#   update: read prims, the V register (or write it), 5 hydro flux components
#           per direction, 3 EMFs; write prims               = 336 B per zone
# (the 2-D geometry tables, 22-62 doubles per (x1, x2) column, amortise over
# the x3 extent and are left out).
FLOPS = {"weno5": {"flux": 1734.0, "update": 1199.8}, "mc": {"flux": 735.3, "update": 1184.3}}
BYTES = {"flux": 128.0, "update": 336.0}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps first (the GPU's clocks settle); the timed steps then "
                         "start again from the initial state")
    ap.add_argument("--n", type=int, default=128, help="zones per axis of the torus")
    ap.add_argument("--recon", choices=("weno5", "mc"), default="weno5")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reduced-precision and batched measurements")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched extra: default tile shapes instead of the autotuner's")
    ap.add_argument("--tune-schedule", action="store_true",
                    help="autotune the x3 run lengths of the single-grid schedule first")
    ap.add_argument("--schedule", default=None,
                    help="KG_FLUX,KG_UPDATE: fixed x3 run lengths of the schedule")
    return ap.parse_args()


_T0 = time.time()


def progress(what):
    """One progress line on stderr per finished part of the run."""
    print(f"[bench] {what} done at {time.time() - _T0:.1f} s", file=sys.stderr, flush=True)


def calibration_copy(torch):
    """One elementwise pass over 512 MiB (read 512 MiB, write 512 MiB) before
    anything else: the reference kernel for scaling the HBM byte counters of a
    profile of this same command."""
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


def oracle_baseline(grid, P, gam, recon, budget_s):
    """The FP64 oracle, as it stands, on all host cores: whole RK2 steps of
    the same grid until about budget_s seconds have passed."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c = oracle.cfg(grid, gam=gam, recon=recon, nthreads=threads)
    nz = grid.n1 * grid.n2 * grid.n3
    steps, t = 0, 0.0
    Q = P
    while t < budget_s and steps < 50:
        t0 = time.perf_counter()
        Q, _, _ = oracle.run(c, Q, -1, 1)
        t += time.perf_counter() - t0
        steps += 1
    out = {"value": nz * steps / t, "unit": "zone-cycles/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} full SSPRK2 step(s) of the same {grid.n1}^3 torus (CFL dt each "
                     f"step), {t:.1f} s wall"}
    # the same on one thread (one step), and the host CPU
    c1 = oracle.cfg(grid, gam=gam, recon=recon, nthreads=1)
    t0 = time.perf_counter()
    oracle.run(c1, P, -1, 1)
    t1 = time.perf_counter() - t0
    out["one_thread_value"] = nz / t1
    out["one_thread_sample"] = f"1 full SSPRK2 step on 1 thread, {t1:.1f} s wall"
    out.update(host_cpu())
    return out


def host_cpu():
    """The host CPU as lscpu reports it (model name, family/model/stepping,
    sockets, cores, threads), and the CPUs this process may run on."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    keys = ("Model name", "Vendor ID", "CPU family", "Model", "Stepping", "Socket(s)",
            "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz")
    out = {"cpu_model": info.get("Model name"),
           "lscpu": {k: info[k] for k in keys if k in info},
           "host_cpus": len(os.sched_getaffinity(0))}
    return out


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(fields["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_source_sha():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2408_01361_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".inc")):
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def _unpack_blocks(flat, blocks):
    """Per-block padded prims (8, n+6, n+6, n+6) out of a pack's flat state."""
    out, o = [], 0
    for b in blocks:
        m = b["n"] + 6
        out.append(flat[o:o + 8 * m ** 3].reshape(8, m, m, m))
        o += 8 * m ** 3
    return out


def time_steps(torch, solver, steps, use_dt=True, dt=None):
    """Wall time of `steps` steps: each at the CFL dt of its input state,
    reduced and applied on the device, or at a fixed dt."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        if use_dt:
            solver.step_cfl()
        else:
            solver.step(dt)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def extras(torch, gr, np, args):
    """Reduced precision (192^3, 50 steps) and batched packs (320 blocks),
    each against plain FP64 on this GPU."""
    from workloads import fm_torus, torus_pack, interior, RECON_WENO5
    from paper_2408_01361_amd import autotune
    out = {}
    gam = 13.0 / 9.0
    n = 192
    grid, P, _ = fm_torus(n, n, n, seed=1, gamma=gam)
    Pt = torch.from_numpy(P).cuda()
    res = {}
    for name, prec in (("fp64", gr.PREC_FP64), ("mixed", gr.PREC_MIXED)):
        s = gr.Grmhd(grid, gam, recon=RECON_WENO5, precision=prec)
        s.load(Pt)
        dt = s.dt()
        if args.tune_schedule:
            autotune.tune_schedule(s, dt)
        for _ in range(10):          # untimed: clocks settle
            s.step(dt)
        s.load(Pt)
        s.reset_status()
        err = {}
        t = 0.0
        done = 0
        for upto in (1, 10, 50):
            t += time_steps(torch, s, upto - done, use_dt=False, dt=dt)
            done = upto
            err[upto] = s.prims().cpu().numpy()
        res[name] = (t, err, s.divb(), s.status()[0])
        del s
    t64, e64, _, _ = res["fp64"]
    t32, e32, divb32, f32 = res["mixed"]
    rel = {}
    for k in (1, 10, 50):
        a, b = interior(e32[k][0]), interior(e64[k][0])
        rel[str(k)] = float(np.abs(a - b).sum() / np.abs(b).sum())
    out["mixed_precision"] = {
        "workload": f"same torus at {n}^3, WENO5, 50 RK2 steps at the initial CFL dt",
        "zone_cycles_per_s": n ** 3 * 50 / t32, "fp64_zone_cycles_per_s": n ** 3 * 50 / t64,
        "speedup_vs_fp64": t64 / t32, "rho_rel_l1_vs_fp64_after_steps": rel,
        "divb_max_mixed": divb32[0], "divb_mean_mixed": divb32[1], "inversion_failures": f32,
        "fp64_reference_note": "the errors are against the FP64 run of this GPU, whose steps match the "
                               "oracle to 1e-12 relative L1 per step at this size (full-size parity tests)"}
    del Pt, res, e64, e32
    progress("mixed precision")
    # batched uneven packs of the 128^3 torus
    g, blocks, _ = torus_pack(nblocks=320, n_global=128, sizes=(16, 32, 64), probs=(0.6, 0.3, 0.1),
                              seed=7, torus_seed=1, gamma=gam)
    flat = torch.from_numpy(np.concatenate([b["prims"].ravel() for b in blocks])).cuda()
    pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], gam, recon=RECON_WENO5)
    pk.load(flat)
    _, Pg, _ = fm_torus(128, 128, 128, seed=1, gamma=gam)
    single = gr.Grmhd(g, gam, recon=RECON_WENO5)
    single.load(torch.from_numpy(Pg).cuda())
    dt = single.dt()
    del single
    tiles = {}
    if not args.no_tune:
        tiles, _ = autotune.tune_pack(pk, dt)
        pk.load(flat)
    zones = sum(b["n"] ** 3 for b in blocks)
    for _ in range(3):               # untimed: clocks settle
        pk.step(dt)
    pk.load(flat)
    torch.cuda.synchronize()
    steps = 10
    f0 = pk.status()
    t0 = time.perf_counter()
    for _ in range(steps):
        pk.step(dt)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    fails = pk.status() - f0
    packed = _unpack_blocks(pk.prims().cpu().numpy(), blocks)
    # the same blocks, each advanced by its own single-grid context (the
    # plain FP64 kernels, one launch sequence per block), one after another
    # on the same stream: the per-block baseline of the batched launch
    ctxs = []
    for b in blocks:
        c = gr.Grmhd(b["grid"], gam, recon=RECON_WENO5)
        c.load(torch.from_numpy(b["prims"]).cuda())
        ctxs.append(c)
    for c in ctxs:                   # untimed: one step each
        c.step(dt)
    for c, b in zip(ctxs, blocks):
        c.load(torch.from_numpy(b["prims"]).cuda())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for c in ctxs:
            c.step(dt)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    num = den = 0.0
    for c, q in zip(ctxs, packed):
        a = interior(c.prims().cpu().numpy())[0]
        num += float(np.abs(interior(q)[0] - a).sum())
        den += float(np.abs(a).sum())
    del ctxs
    out["batched"] = {
        "workload": "320 frozen-ghost blocks of the 128^3 torus, n in {16,32,64} (60/30/10 %, seed 7), "
                    "WENO5, FP64, three launches per RK2 stage (fluxes, EMFs, update) over all blocks, "
                    "10 steps at fixed dt",
        "interior_zones": zones, "zone_cycles_per_s": zones * steps / tp,
        "per_block_zone_cycles_per_s": zones * steps / tb,
        "speedup_vs_per_block_fp64": tb / tp,
        "rho_rel_l1_vs_per_block_fp64": num / den,
        "per_block_note": "the same blocks and steps, each block its own single-grid FP64 context "
                          "stepped in turn on one stream (one ctypes call and its launches per "
                          "block and step)",
        "workgroups_per_stage": pk.grid_blocks,
        "tiles": {str(k): list(v) for k, v in tiles.items()},
        "tiles_note": "per block size: t1 x t2 x t3 zones, or [0, 0, 0] = runs of 256 consecutive "
                      "positions of each box",
        "inversion_failures_timed_steps": fails}
    progress("batched pack")
    out["tiling_exchange"] = tiling_extra(torch, gr, np, gam, dt, steps, args)
    progress("tiling with ghost exchange")
    out["adjoint"] = adjoint_extra(torch, gr)
    return out


def tiling_extra(torch, gr, np, gam, dt, steps, args):
    """The whole 128^3 torus as an uneven octree-like tiling (blocks of 16,
    32 and 64) advanced as one pack with the ghost exchange before every
    stage, against the single 128^3 grid at the same fixed dt: throughput of
    both and the density L1 of the tiling against the grid after the steps."""
    from workloads import torus_tiling, interior, RECON_WENO5
    from paper_2408_01361_amd import autotune
    g, blocks, P, _ = torus_tiling(128, sizes=(16, 32, 64), split=0.6, seed=5, gamma=gam)
    flat = torch.from_numpy(np.concatenate([b["prims"].ravel() for b in blocks])).cuda()
    pk = gr.Pack(g, [b["n"] for b in blocks], [b["offset"] for b in blocks], gam, recon=RECON_WENO5)
    pk.set_exchange(True)
    pk.load(flat)
    if not args.no_tune:
        autotune.tune_pack(pk, dt)
        pk.load(flat)
    for _ in range(3):               # untimed: clocks settle
        pk.step(dt)
    pk.load(flat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pk.step(dt)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    packed = _unpack_blocks(pk.prims().cpu().numpy(), blocks)
    fails_pack = pk.status()
    pk.set_exchange(False)           # the same pack with frozen ghosts: the exchange's cost
    pk.load(flat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pk.step(dt)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    del pk, flat
    s = gr.Grmhd(g, gam, recon=RECON_WENO5)
    Pt = torch.from_numpy(P).cuda()
    s.load(Pt)
    for _ in range(3):
        s.step(dt)
    s.load(Pt)
    s.reset_status()
    ts = time_steps(torch, s, steps, use_dt=False, dt=dt)
    ref = interior(s.prims().cpu().numpy())[0]
    fails_single = s.status()[0]
    num = 0.0
    for b, q in zip(blocks, packed):
        i, j, k = b["offset"]
        n = b["n"]
        num += float(np.abs(interior(q)[0] - ref[k:k + n, j:j + n, i:i + n]).sum())
    zones = 128 ** 3
    counts = ", ".join(f"{sum(1 for b in blocks if b['n'] == m)} x {m}^3" for m in (16, 32, 64))
    return {"workload": f"128^3 torus tiled by {len(blocks)} blocks ({counts}), WENO5, FP64, "
                        f"ghost exchange + three launches per stage over all blocks, {steps} steps at fixed dt",
            "zone_cycles_per_s": zones * steps / tp,
            "frozen_ghosts_zone_cycles_per_s": zones * steps / tf,
            "single_grid_zone_cycles_per_s": zones * steps / ts,
            "rho_rel_l1_vs_single_grid": num / float(np.abs(ref).sum()),
            "inversion_failures": {"tiling": fails_pack, "single_grid": fails_single}}


def kastaun_extra(torch, gr, grid, P, gam, recon, steps):
    """The headline workload with the Kastaun et al. bracketed recovery and
    with the implicit solver's Newton in place of 1D_W, each timed the same
    way (whole steps, then the update classes, which hold the inversion --
    for the implicit recovery the update that stores U* plus the solver's
    own pass -- with per-launch events)."""
    Pt = torch.from_numpy(P).cuda()
    res = {}
    for name, inv in (("1dw", gr.INV_1DW), ("kastaun", gr.INV_KASTAUN), ("implicit", gr.INV_IMPLICIT)):
        s = gr.Grmhd(grid, gam, recon=recon, inverter=inv)
        s.load(Pt)
        for _ in range(10):          # untimed: clocks settle
            s.step_cfl()
        s.load(Pt)
        s.reset_status()
        el = time_steps(torch, s, steps)
        fails = s.status()[0]
        s.load(Pt)
        s.timing(True, classes=["update1", "update2"])
        time_steps(torch, s, steps)
        rep = s.timing_report()
        s.timing(False)
        res[name] = {"zone_cycles_per_s": grid.n1 * grid.n2 * grid.n3 * steps / el,
                     "ms_per_step": el * 1e3 / steps,
                     "update_us_per_step": {k: 1e3 * rep[k][0] / steps for k in ("update1", "update2")},
                     "inversion_failures": fails}
        del s
    res["workload"] = "the headline torus and step, inverter swapped"
    res["kastaun_over_1dw_time"] = res["kastaun"]["ms_per_step"] / res["1dw"]["ms_per_step"]
    res["implicit_over_1dw_time"] = res["implicit"]["ms_per_step"] / res["1dw"]["ms_per_step"]
    return res


def recon_extra(torch, gr, grid, P, gam, steps):
    """The headline torus and step with each reconstruction: whole steps
    (CFL dt each step) and the flux class (both stages) with per-launch
    events; FP64 and, for each, the mixed-precision form."""
    Pt = torch.from_numpy(P).cuda()
    res = {}
    names = (("donor", gr.RECON_DONOR), ("mc", gr.RECON_MC), ("vl", gr.RECON_VL),
             ("ppm", gr.RECON_PPM), ("ppmx", gr.RECON_PPMX), ("mp5", gr.RECON_MP5), ("weno5", gr.RECON_WENO5),
             ("wenoz", gr.RECON_WENOZ))
    for name, recon in names:
        row = {}
        for pname, prec in (("fp64", gr.PREC_FP64), ("mixed", gr.PREC_MIXED)):
            s = gr.Grmhd(grid, gam, recon=recon, precision=prec)
            s.load(Pt)
            for _ in range(10):          # untimed: clocks settle
                s.step_cfl()
            s.load(Pt)
            el = time_steps(torch, s, steps)
            s.load(Pt)
            s.timing(True, classes=["flux"])
            time_steps(torch, s, steps)
            rep = s.timing_report()
            s.timing(False)
            row[pname] = {"zone_cycles_per_s": grid.n1 * grid.n2 * grid.n3 * steps / el,
                          "ms_per_step": el * 1e3 / steps,
                          "flux_us_per_step": 1e3 * rep["flux"][0] / steps}
            del s
        res[name] = row
    res["workload"] = "the headline torus and step, reconstruction swapped"
    return res


def integrator_extra(torch, gr, grid, P, gam, recon, steps):
    """The headline torus and step with each time integrator (CFL dt each
    step): SSPRK2, predictor-corrector, RK1, SSPRK(5,4)."""
    Pt = torch.from_numpy(P).cuda()
    res = {}
    for name, integ in (("ssprk2", gr.INTEG_SSPRK2), ("pc", gr.INTEG_PC), ("rk1", gr.INTEG_RK1),
                        ("ssprk54", gr.INTEG_SSPRK54)):
        s = gr.Grmhd(grid, gam, recon=recon, integrator=integ)
        s.load(Pt)
        for _ in range(10):          # untimed: clocks settle
            s.step_cfl()
        s.load(Pt)
        el = time_steps(torch, s, steps)
        res[name] = {"zone_cycles_per_s": grid.n1 * grid.n2 * grid.n3 * steps / el,
                     "ms_per_step": el * 1e3 / steps}
        del s
    res["workload"] = ("the headline torus and step, integrator swapped (a step of RK1 is one stage, "
                       "of SSPRK(5,4) five)")
    return res


def egrmhd_extra(torch, gr, grid, P, gam, recon, steps):
    """Extended GRMHD against the ideal step on the headline torus: the
    predictor-corrector with the 1D_W recovery (the ideal step of the same
    integrator), SSPRK2 with the implicit solver's Newton as the recovery
    (the same per-zone solver without the extra variables), and Extended
    GRMHD (predictor-corrector; heat flux and pressure anisotropy, tau_R = 1,
    chi = nu = 0.1, from zero extra variables).  CFL dt each step."""
    Pt = torch.from_numpy(P).cuda()
    nz = grid.n1 * grid.n2 * grid.n3
    res = {}
    for name, kw in (("ideal_pc_1dw", dict(integrator=gr.INTEG_PC)),
                     ("ideal_ssprk2_implicit", dict(inverter=gr.INV_IMPLICIT)),
                     ("egrmhd", dict(integrator=gr.INTEG_PC, egrmhd=True, tau_r=1.0, chi_emhd=0.1,
                                     nu_emhd=0.1))):
        s = gr.Grmhd(grid, gam, recon=recon, **kw)
        s.load(Pt)
        for _ in range(3):           # untimed: clocks settle
            s.step_cfl()
        s.load(Pt)
        if name == "egrmhd":
            s.load_extended(torch.zeros((2,) + tuple(Pt.shape[1:]), dtype=torch.float64, device="cuda"))
        s.reset_status()
        el = time_steps(torch, s, steps)
        res[name] = {"zone_cycles_per_s": nz * steps / el, "ms_per_step": el * 1e3 / steps,
                     "failed_zone_solves": s.status()[0]}
        s.close()
    res["slowdown_vs_ideal_pc"] = res["ideal_pc_1dw"]["zone_cycles_per_s"] / res["egrmhd"]["zone_cycles_per_s"]
    res["slowdown_vs_ideal_ssprk2_implicit"] = (res["ideal_ssprk2_implicit"]["zone_cycles_per_s"] /
                                                res["egrmhd"]["zone_cycles_per_s"])
    res["workload"] = ("the headline torus, predictor-corrector; Extended GRMHD with tau_R = 1, "
                       "chi = nu = 0.1, no floors (failed zone solves keep their state)")
    return res


def floors_fofc_extra(torch, gr, grid, P, gam, recon, steps):
    """What the floors and the first-order flux correction cost: the headline
    torus step plain, with floors, with floors plus the correction, and with
    both and the Kastaun recovery (the production settings); and
    the magnetised blast at 1024^2 (flat space), where the correction acts,
    without and with it (failed inversions and marked zones per run)."""
    from workloads import magnetised_blast, RECON_MC
    out = {}
    Pt = torch.from_numpy(P).cuda()
    torus = {}
    for name, kw in (("plain", {}), ("floors", dict(floors=True)),
                     ("floors_fofc", dict(floors=True, fofc=True)),
                     ("kastaun_floors_fofc", dict(floors=True, fofc=True, inverter=gr.INV_KASTAUN))):
        s = gr.Grmhd(grid, gam, recon=recon, **kw)
        s.load(Pt)
        for _ in range(10):          # untimed: clocks settle
            s.step_cfl()
        s.load(Pt)
        s.reset_status()
        el = time_steps(torch, s, steps)
        torus[name] = {"zone_cycles_per_s": grid.n1 * grid.n2 * grid.n3 * steps / el,
                       "ms_per_step": el * 1e3 / steps, "counters": s.counters()}
        del s
    torus["workload"] = "the headline torus and step"
    out["torus"] = torus
    del Pt
    n, nsteps = 1024, 20
    bg, bP = magnetised_blast(n)
    bPt = torch.from_numpy(bP).cuda()
    blast = {}
    for name, kw in (("plain", {}), ("fofc", dict(fofc=True)), ("floors_fofc", dict(floors=True, fofc=True))):
        s = gr.Grmhd(bg, 4.0 / 3.0, recon=RECON_MC, **kw)
        s.load(bPt)
        for _ in range(5):
            s.step_cfl()
        s.load(bPt)
        s.reset_status()
        el = time_steps(torch, s, nsteps)
        blast[name] = {"zone_cycles_per_s": n * n * nsteps / el, "ms_per_step": el * 1e3 / nsteps,
                       "counters": s.counters()}
        del s
    blast["workload"] = (f"magnetised cylindrical explosion, flat, {n}^2 x 1, MC, FP64, {nsteps} RK2 "
                         "steps at the CFL dt from the initial state")
    out["blast"] = blast
    return out


def face_ct_extra(torch, gr, grid, P, info, gam, recon, steps):
    """The headline torus step with face-centred CT (averaged and upwinded
    edge EMFs) beside Flux-CT: whole steps, then a per-class breakdown."""
    Pt = torch.from_numpy(P).cuda()
    Ft = torch.from_numpy(info["faces"]).cuda()
    res = {}
    for name, ct in (("flux_ct", gr.CT_FLUX), ("face_avg", gr.CT_FACE_AVG), ("face_gs", gr.CT_FACE_GS)):
        s = gr.Grmhd(grid, gam, recon=recon, ct=ct)

        def load():
            s.load(Pt)
            if ct != gr.CT_FLUX:
                s.load_faces(Ft)
        load()
        for _ in range(10):          # untimed: clocks settle
            s.step_cfl()
        load()
        el = time_steps(torch, s, steps)
        load()
        s.timing(True)
        time_steps(torch, s, steps)
        rep = s.timing_report()
        s.timing(False)
        res[name] = {"zone_cycles_per_s": grid.n1 * grid.n2 * grid.n3 * steps / el,
                     "ms_per_step": el * 1e3 / steps,
                     "kernels_us_per_step": {k: round(1e3 * v[0] / steps, 1) for k, v in rep.items() if v[1]}}
        if ct != gr.CT_FLUX:
            res[name]["face_divb_max"] = s.face_divb()[0]
        del s
    res["workload"] = "the headline torus and step; face fields from the same vector potential"
    return res


def timing_protocol_extra(torch, gr, grid, P, gam, recon, steps):
    """The headline step timed as repeated runs: the median over 5 repeats
    of the K steps (each from the reloaded initial state), with the device
    CFL reduction and with a fixed dt (no reduction); and the small
    workload (fast mode, 32^3, MC), launch-bound, over 1000 steps."""
    import numpy as np
    from workloads import linear_mode, RECON_MC
    Pt = torch.from_numpy(P).cuda()
    s = gr.Grmhd(grid, gam, recon=recon)
    s.load(Pt)
    dt = s.dt()
    for _ in range(10):
        s.step_cfl()
    reps = {"cfl": [], "fixed_dt": []}
    for _ in range(5):
        s.load(Pt)
        reps["cfl"].append(time_steps(torch, s, steps) * 1e3 / steps)
        s.load(Pt)
        reps["fixed_dt"].append(time_steps(torch, s, steps, use_dt=False, dt=dt) * 1e3 / steps)
    del s
    out = {k: {"median_ms_per_step": float(np.median(v)), "min": min(v), "max": max(v)} for k, v in reps.items()}
    out["workload"] = "the headline torus and step, 5 repeats of the K steps"
    g, Pm, _, _ = linear_mode("fast", 32, ndim=3)
    sm = gr.Grmhd(g, 4.0 / 3.0, recon=RECON_MC)
    sm.load(torch.from_numpy(Pm).cuda())
    for _ in range(50):
        sm.step_cfl()
    el = time_steps(torch, sm, 1000)
    out["fast_mode_32"] = {"workload": "fast mode, flat periodic 32^3, MC, FP64, 1000 CFL steps",
                           "zone_cycles_per_s": 32 ** 3 * 1000 / el, "us_per_step": el * 1e6 / 1000}
    return out


def adjoint_extra(torch, gr):
    """Gradient of sum_{i<5} rho u after 8 steps of the 64^3 torus (MC, FP64,
    fixed dt) with respect to the initial prims and gamma: the forward pass
    with per-step checkpoints and the hand-written backward, timed apart."""
    from workloads import fm_torus, RECON_MC, NG
    from paper_2408_01361_amd import autograd as ag
    gam, n, nsteps = 13.0 / 9.0, 64, 8
    grid, P, _ = fm_torus(n, n, n, seed=1, gamma=gam)
    s = gr.Grmhd(grid, gam, recon=RECON_MC)
    Pt = torch.from_numpy(P).cuda()
    s.load(Pt)
    dt = s.dt()

    def one():
        x = Pt.clone().requires_grad_(True)
        gt = torch.tensor(gam, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ag.run(x, gt, s, dt, nsteps)
        I = out[:, NG:-NG, NG:-NG, NG:-NG]
        L = (I[0, :, :, :5] * I[1, :, :, :5]).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    one()                            # untimed: workspaces, clocks
    runs = [one() for _ in range(3)]
    tf, tb = min(r[0] for r in runs), min(r[1] for r in runs)
    zc = n ** 3 * nsteps
    return {"workload": "64^3 torus, MC, FP64, 8 RK2 steps at fixed dt, loss sum_{i<5} rho u; "
                        "gradient in the initial prims and gamma (best of 3)",
            "forward_ms_per_step": tf * 1e3 / nsteps, "backward_ms_per_step": tb * 1e3 / nsteps,
            "backward_over_forward": tb / tf, "gradient_zone_cycles_per_s": zc / (tf + tb)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; runs on several GPUs are not "
                                   "part of it (use --gpus 1)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from workloads import fm_torus, RECON_MC, RECON_WENO5
    from paper_2408_01361_amd import grmhd as gr
    from paper_2408_01361_amd import autotune

    n = args.n
    gam = 13.0 / 9.0
    recon = RECON_WENO5 if args.recon == "weno5" else RECON_MC
    grid, P, info = fm_torus(n, n, n, seed=1, gamma=gam)
    calibration_copy(torch)
    Pt = torch.from_numpy(P).cuda()
    s = gr.Grmhd(grid, gam, recon=recon, precision=gr.PREC_FP64)
    s.load(Pt)
    sched = None
    if args.schedule:
        sched = tuple(int(x) for x in args.schedule.split(","))
        s.set_schedule(*sched)
    elif args.tune_schedule:
        sched, _ = autotune.tune_schedule(s, s.dt())
        s.load(Pt)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        s.step_cfl()
    # per-class breakdown: the same K steps with every kernel class timed
    s.load(Pt)
    s.timing(True)
    time_steps(torch, s, args.steps)
    rep = s.timing_report()
    s.timing(False)
    cls = {k: v for k, v in rep.items() if v[1] > 0}
    dom = max(cls, key=lambda k: cls[k][0])
    # the timed region: steps 1..K of the workload; only the dominant class's
    # launches carry timing events (they travel in the dispatches themselves)
    s.load(Pt)
    s.reset_status()
    s.timing(True, classes=[dom])
    el = time_steps(torch, s, args.steps)
    rep_dom = s.timing_report()
    s.timing(False)
    fails = s.status()[0]
    nz = n ** 3
    ms_step = el * 1e3 / args.steps
    zcps = nz * args.steps / el

    # roofline of the dominant kernel class, from the timed region's events
    ms, launches = rep_dom[dom]
    avg_s = ms * 1e-3 / launches
    kind = "flux" if dom == "flux" else ("update" if dom.startswith("update") else None)
    roof = {"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None,
            "kernel": dom, "avg_us": avg_s * 1e6}
    if kind:
        # one flux launch evaluates the x1, x2 and x3 faces of the flux boxes
        units = 3 * (n + 1) * (n + 2) * (n + 2) if kind == "flux" else nz
        flops = FLOPS[args.recon][kind] * units
        nbytes = BYTES[kind] * units
        f_alu = flops / avg_s / 1e12 / PEAK_FP64_TFLOPS
        f_hbm = nbytes / avg_s / 1e9 / PEAK_HBM_GBS
        if f_alu >= f_hbm:
            roof.update(bound="alu", achieved=flops / avg_s / 1e12, peak=PEAK_FP64_TFLOPS,
                        unit="TFLOP/s", frac=f_alu)
        else:
            roof.update(bound="hbm", achieved=nbytes / avg_s / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                        frac=f_hbm)
        roof["algorithmic_flops_per_launch"] = flops
        roof["algorithmic_bytes_per_launch"] = nbytes
        roof["hbm_frac_algorithmic"] = f_hbm
        roof["traffic"] = traffic_from_profile(dom, f"torus{n}_{args.recon}")
    # breakdown pass (all classes timed; same steps, outside the timed region)
    kernels = {k: {"ms_total": round(v[0], 4), "launches": v[1],
                   "avg_us": round(1e3 * v[0] / max(v[1], 1), 2)} for k, v in rep.items()}
    out = {
        "metric": "zone-cycles/sec per RK2 step (FP64 vs mixed vs batched) + % HBM roofline",
        "value": zcps,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"magnetised FM torus, Kerr a=0.9375 MKS h=0.3, {n}^3, "
                               f"{args.recon.upper()}, FP64, SSPRK2 + LLF + Flux-CT + 1D_W, CFL dt "
                               f"each step", "zones": nz, "gamma_ad": gam, "seed": 1,
                   "inversion_failures": fails, "schedule_kg": sched},
        "roofline": roof,
        "kernels": kernels,
        # whole step against HBM: the method's minimum (read and write the 8-variable
        # state and the stage register: 6 x 64 B per zone-cycle) and this design's
        # kernel sequence (2 stages x (3 flux passes + update))
        "hbm_frac_step_min_384B": zcps * 384.0 / 1e9 / PEAK_HBM_GBS,
        "hbm_frac_step_design_bytes": zcps * 2 * (3 * BYTES["flux"] + BYTES["update"]) / 1e9 / PEAK_HBM_GBS,
    }
    # the headline fractions by name: which roof binds the dominant kernel, its
    # FP64-ALU and HBM fractions, and the whole step against the HBM roof
    if kind:
        out["headline_fractions"] = {
            "dominant_kernel": dom,
            "binding_roof": "fp64_alu" if roof["bound"] == "alu" else "hbm",
            "dominant_kernel_alu_frac": f_alu,
            "dominant_kernel_hbm_frac": f_hbm,
            "step_hbm_frac_min_384B": out["hbm_frac_step_min_384B"],
            "step_hbm_frac_60pct_target_met": out["hbm_frac_step_min_384B"] >= 0.6,
        }
    s.close()
    progress("headline")
    if not args.no_extras:
        out.update(extras(torch, gr, np, args))
        progress("adjoint")
        legs = (("inverters", lambda: kastaun_extra(torch, gr, grid, P, gam, recon, args.steps)),
                ("reconstructions", lambda: recon_extra(torch, gr, grid, P, gam, args.steps)),
                ("integrators", lambda: integrator_extra(torch, gr, grid, P, gam, recon, args.steps)),
                ("egrmhd", lambda: egrmhd_extra(torch, gr, grid, P, gam, recon, args.steps)),
                ("floors_fofc", lambda: floors_fofc_extra(torch, gr, grid, P, gam, recon, args.steps)),
                ("face_ct", lambda: face_ct_extra(torch, gr, grid, P, info, gam, recon, args.steps)),
                ("timing_protocol", lambda: timing_protocol_extra(torch, gr, grid, P, gam, recon, args.steps)))
        for name, leg in legs:
            out[name] = leg()
            progress(name)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_baseline(grid, P, gam, recon, args.cpu_seconds)
        progress("cpu baseline")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
