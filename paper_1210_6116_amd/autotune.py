"""Tile-height autotuner: times the sweep of a given replica set on the device
for each tile height (64 x 16, 64 x 32, 64 x 64 tiles) and keeps the fastest.

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
