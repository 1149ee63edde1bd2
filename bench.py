"""Throughput of the HARM ideal-GRMHD step on one MI355X.

Workload (default): the magnetised Fishbone-Moncrief torus in Kerr a = 0.9375,
modified Kerr-Schild coordinates (h = 0.3, r from 0.95 r+ to 1000), r_in = 6,
r_max = 12, gamma = 13/9, beta_min = 100, u perturbed by +-4 % (seed 1),
128^3 zones, WENO5, FP64.  A step is one SSPRK2 step (both stages: ghost
fill, reconstruction + face states + LLF fluxes along x1..x3, Flux-CT EMFs,
divergence + source + RK combine + 1D_W inversion) plus the CFL dt
reduction that chooses it.  Inputs are resident in HBM before timing starts.

Prints one JSON line: zone-cycles per second, the roofline of the dominant
kernel (its time from HIP events recorded on the library's stream during the
timed region), and the FP64 CPU oracle timed on a bounded sample.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks used for the roofline fraction.
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3

# Algorithmic cost per unit of the per-class kernels: bytes that must cross
# HBM at least once, and flops counted by the oracle's counting build
# (oracle/count_flops.py; every +, -, *, /, sqrt is one flop).  A flux unit is
# one face, an update unit one zone.
FLOPS_PER_FACE = {("weno5", "fp64"): None, ("mc", "fp64"): None}
FLOPS_PER_ZONE_UPDATE = None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="zones per axis of the torus")
    ap.add_argument("--recon", choices=("weno5", "mc"), default="weno5")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def oracle_baseline(grid, P, gam, recon, budget_s):
    """The FP64 oracle, as it stands, on all host cores: whole RK2 steps of
    the same grid until about budget_s seconds have passed."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    c = oracle.cfg(grid, gam=gam, recon=recon, nthreads=threads)
    nz = grid.n1 * grid.n2 * grid.n3
    dt = oracle.estimate_dt(c, P)
    steps, t = 0, 0.0
    Q = P
    while t < budget_s and steps < 50:
        t0 = time.perf_counter()
        Q, _, _ = oracle.run(c, Q, -1, 1)
        t += time.perf_counter() - t0
        steps += 1
    return {"value": nz * steps / t, "unit": "zone-cycles/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} full SSPRK2 step(s) of the same {grid.n1}x{grid.n2}x{grid.n3} "
                      f"torus with per-step CFL dt, {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part "
                                   "of it (pass --gpus 1)"}))
        sys.exit(2)
    import numpy as np
    import torch
    from workloads import fm_torus, RECON_MC, RECON_WENO5
    from paper_2408_01361_amd import grmhd as gr

    n = args.n
    gam = 13.0 / 9.0
    recon = RECON_WENO5 if args.recon == "weno5" else RECON_MC
    prec = gr.PREC_FP64 if args.precision == "fp64" else gr.PREC_MIXED
    grid, P, info = fm_torus(n, n, n, seed=1, gamma=gam)
    s = gr.Grmhd(grid, gam, recon=recon, precision=prec)
    s.load(torch.from_numpy(P).cuda())
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        s.step(s.dt())
    torch.cuda.synchronize()

    s.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step(s.dt())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = s.timing_report()
    s.timing(False)
    fails = s.status()[0]

    nz = n ** 3
    ms_step = (t1 - t0) * 1e3 / args.steps
    zcps = nz * args.steps / (t1 - t0)

    # dominant kernel class by event time
    dom = max(rep, key=lambda k: rep[k][0])
    dom_ms, dom_launches = rep[dom]
    avg_ms = dom_ms / max(dom_launches, 1)
    kernels = {k: {"ms_total": round(v[0], 4), "launches": v[1],
                   "avg_us": round(1e3 * v[0] / max(v[1], 1), 2)} for k, v in rep.items()}
    roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": None, "traffic": None, "kernel": dom, "avg_us": round(1e3 * avg_ms, 2)}

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
        "dtype": "f64" if prec == gr.PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"magnetised FM torus, Kerr a=0.9375 MKS, {n}^3, "
                               f"{args.recon.upper()}, {args.precision}, SSPRK2 + 1D_W + Flux-CT",
                   "zones": nz, "gamma_ad": gam, "seed": 1, "inversion_failures": fails},
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_baseline(grid, P, gam, recon, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
