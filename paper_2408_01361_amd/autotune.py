"""Autotuner for launch shapes: pack tile shapes per block size, and the x3
run length of the single-block schedule.

Candidates are timed on the live object with HIP events (torch.cuda.Event on
the object's stream) and the fastest is kept.  Results are cached as JSON
(keyed by GPU architecture, reconstruction, precision and size) under
$XDG_CACHE_HOME/grmhd or ~/.cache/grmhd; a cached entry is reused without
timing.  Launch shapes never change results, only speed.
"""

import json
import os

import torch

# (0, 0, 0): linear runs of 256 consecutive positions of each box
TILE_CANDIDATES = [(0, 0, 0), (64, 4, 1), (32, 8, 1), (16, 16, 1), (16, 8, 2), (8, 8, 4), (32, 4, 2),
                   (16, 4, 4), (8, 4, 8), (4, 8, 8), (128, 2, 1), (64, 2, 2)]
KG_CANDIDATES = [1, 2, 4, 8, 16, 32]


def _cache_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "grmhd", "autotune.json")


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _time(fn, stream, reps):
    fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        for _ in range(reps):
            fn()
        end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps


def tune_pack(pack, dt, reps=3, rounds=1, use_cache=True):
    """Coordinate search over tile shapes, one block size at a time.  The
    pack's state advances while timing: load it again afterwards."""
    cache = _load() if use_cache else {}
    key = lambda n: f"{_arch()}|pack|recon{pack.params.recon}|fp64|n{n}"
    sizes = sorted(set(pack.sizes))
    chosen = {}
    todo = []
    for n in sizes:
        if key(n) in cache:
            chosen[n] = tuple(cache[key(n)])
            pack.set_tiles(n, *chosen[n])
        else:
            todo.append(n)
    timings = {}
    for _ in range(rounds):
        for n in todo:
            best = None
            for t in TILE_CANDIDATES:
                if t[0] > 2 * (n + 2) or t[1] > 2 * (n + 2) or t[2] > 2 * (n + 2):
                    continue
                pack.set_tiles(n, *t)
                ms = _time(lambda: pack.step(dt), pack.stream, reps)
                timings[(n, t)] = ms
                if best is None or ms < best[0]:
                    best = (ms, t)
            chosen[n] = best[1]
            pack.set_tiles(n, *best[1])
    cache = _load()
    for n in todo:
        cache[key(n)] = list(chosen[n])
    if todo and use_cache:
        _save(cache)
    return chosen, timings


def tune_schedule(solver, dt, reps=3, use_cache=True):
    """x3 run length of the flux/EMF and update schedules of one context."""
    g = solver.spec
    key = f"{_arch()}|single|recon{solver.params.recon}|prec{solver.params.precision}|{g.n1}x{g.n2}x{g.n3}"
    cache = _load() if use_cache else {}
    if key in cache:
        kf, ku = cache[key]
        solver.set_schedule(kf, ku)
        return (kf, ku), {}
    timings = {}
    best = None
    for kg in KG_CANDIDATES:
        solver.set_schedule(kg, kg)
        ms = _time(lambda: solver.step(dt), solver.stream, reps)
        timings[kg] = ms
        if best is None or ms < best[0]:
            best = (ms, kg)
    solver.set_schedule(best[1], best[1])
    if use_cache:
        cache = _load()
        cache[key] = [best[1], best[1]]
        _save(cache)
    return (best[1], best[1]), timings
