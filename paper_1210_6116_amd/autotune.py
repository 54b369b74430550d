"""Autotuner of the sweep's shape choices, timed on the device for a given
replica set: the tile height (64 x 16, 64 x 32, 64 x 64 tiles; tune), then
the merge schedule (tune_merge): the merge's pair deduplication and the tile
edges each of its waves unites.  None of the choices changes a result, only
the speed.

Results are cached as JSON (keyed by the replica sizes, the label width and the
GPU architecture) under $XDG_CACHE_HOME/xymc (default ~/.cache/xymc).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

CANDIDATES = (16, 32, 64)


def _cache_path():
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "xymc", "autotune.json")


def _key(specs, arch):
    sizes = sorted(int(s["L"]) for s in specs)
    h = hashlib.sha1(json.dumps(sizes).encode()).hexdigest()[:16]
    bits = 64 if max(sizes) ** 2 >= 2 ** 32 else 32
    return "%s/%d/%s/n%d" % (arch, bits, h, len(sizes))


def tile_rows(specs, sweeps: int = 20, warmup: int = 5, use_cache: bool = True) -> int:
    """Fastest tile height for these replicas (a list of dicts with L, beta, seed)."""
    return tune(specs, sweeps, warmup, use_cache)[0]


def tune(specs, sweeps: int = 20, warmup: int = 5, use_cache: bool = True):
    """(fastest tile height, {tile height: seconds per sweep}) for these replicas;
    the timings are those of the run that chose it (from the cache if present)."""
    from . import Lattices

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = _key(specs, arch)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            rec = cache[key]
            return int(rec["tile_rows"]), {int(k): v * 1e-3 for k, v in rec["ms_per_sweep"].items()}
    timings = {}
    label64 = max(int(s["L"]) for s in specs) ** 2 >= 2 ** 32
    for rows in CANDIDATES:
        if label64 and rows > 32:
            continue
        lat = Lattices([dict(s, tile_rows=rows) for s in specs])
        lat.sweep(warmup)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lat.sweep(sweeps)
        torch.cuda.synchronize()
        timings[rows] = (time.perf_counter() - t) / sweeps
        lat.close()
        del lat
    best = min(timings, key=timings.get)
    cache[key] = dict(tile_rows=best, ms_per_sweep={str(k): v * 1e3 for k, v in timings.items()})
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    return best, timings


def merge_candidates():
    """The merge schedules timed: (pair deduplication, tile edges per wave, 0)
    for the merge kernel, and (hash deduplication, 1, 1) for the merge inside
    the labelling tile pass."""
    from . import _lib

    return [(dd, epw, 0) for dd in (_lib.XY_DEDUP_WAVE, _lib.XY_DEDUP_NEIGHBOUR, _lib.XY_DEDUP_HASH)
            for epw in (1, 2, 4)] + [(_lib.XY_DEDUP_HASH, 1, 1)]


def tune_merge(specs, rows: int, sweeps: int = 50, warmup: int = 200, repeats: int = 3, use_cache: bool = True,
               step=None, tag: str = ""):
    """((dedup, edges per wave, in pass) fastest for these replicas at this tile
    height, {choice: seconds per sweep}); cached like the tile height.

    The choices are timed on one handle, thermalised by `warmup` sweeps first
    (the forest's shape, and with it the merge and the edge coins, depends on
    the state: a hot start ranks the choices differently), switching the
    schedule between blocks of `sweeps` sweeps, `repeats` rounds over all
    choices; a choice's time is its fastest block.  step(lat, n): how n sweeps
    of the workload are run (default: plain sweeps; a PCC run passes its own
    call, since its window ends run other tile passes); tag names it in the
    cache key."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = _key(specs, arch) + "/rows%d/merge2" % rows + ("/" + tag if tag else "")
    if step is None:
        def step(lat, n):
            lat.sweep(n)
    path = _cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        rec = cache[key]
        timings = {tuple(int(x) for x in k.split(",")): v * 1e-3 for k, v in rec["ms_per_sweep"].items()}
        return (int(rec["dedup"]), int(rec["edges_per_wave"]), int(rec["in_pass"])), timings
    from . import Lattices

    lat = Lattices([dict(s, tile_rows=rows) for s in specs])
    step(lat, warmup)
    timings = {}
    for _ in range(repeats):
        for choice in merge_candidates():
            configure(lat, choice)
            torch.cuda.synchronize()
            t = time.perf_counter()
            step(lat, sweeps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / sweeps
            timings[choice] = min(dt, timings.get(choice, dt))
    lat.close()
    best = min(timings, key=timings.get)
    cache[key] = dict(dedup=best[0], edges_per_wave=best[1], in_pass=best[2],
                      ms_per_sweep={"%d,%d,%d" % k: v * 1e3 for k, v in timings.items()})
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1)
    except OSError:
        pass
    return best, timings


def configure(lat, choice):
    """Applies a (dedup, edges per wave, in pass) choice of tune_merge to a handle."""
    lat.set_merge(choice[0], choice[1])
    lat.set_merge_in_pass(bool(choice[2]) if len(choice) > 2 else False)
