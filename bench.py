#!/usr/bin/env python3
"""Throughput of Swendsen-Wang sweeps of the 2D XY model on one MI355X.

Metric: spin updates per second = sweeps x L^2 / wall time.  The headline
workload is a single L = 4096 lattice at beta = 1.12 from a uniform-angle hot
start: 200 thermalisation sweeps (always, untimed) and `--warmup` more untimed
sweeps, then exactly `--steps` sweeps timed between two device
synchronisations.  A "step" is one full sweep: mirror direction, link
activation, labelling, cluster reflection and the observable reductions.

A second, instrumented pass of the same length records HIP events on the
handle's stream around every kernel launch and every sweep; it gives the
per-kernel average durations (roofline of the dominant kernel) and the
per-sweep p50 / p99 latency.  The CPU oracle is timed on 20 sweeps of the
GPU's thermalised lattice on this host (cpu_baseline).  The other workloads
(L = 65536 PCC run, 512-replica batch against plain handles, the serving
trace against one-request-at-a-time plain runs) run at their full shapes
unless cut down by flags; a leg that would run past --time-budget seconds of
bench time is skipped (and says so), and the sequential serving leg starts no
request after it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
THERM_SWEEPS = 200     # thermalisation of the L = 4096 workload before any timing
# Algorithmic bytes per spin update of one sweep with the fewest passes the
# layout of the workloads allows: read labels + read spins + write spins +
# write labels = 4 + 8 + 8 + 4 (32-bit labels), 8 + 8 + 8 + 8 (64-bit labels)
SWEEP_BYTES = {32: 24.0, 64: 32.0}
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz; a wave64 VALU
# instruction occupies its SIMD for 4 cycles (= 39.3e12 lane-instructions/s)
VALU_PEAK_TLANE = 256 * 4 * 16 * 2.4e9 / 1e12
# device code of the sweep kernels: the counter file is valid only for these exact sources
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1210_6116_amd", "csrc", f)
                  for f in ("xy_kernels.hip", "xy_device.hpp", "xy_launch.hpp")] + [
                     os.path.join(ROOT, "include", "xy.h")]
COUNTERS = os.path.join(ROOT, "profiles", "counters_L4096.json")


def alg_bytes_per_site(kernel: str, tile_rows: int = 32) -> float:
    """Algorithmic HBM bytes per site of one launch of each kernel (64-column
    tiles of tile_rows rows; labels are 16-bit and tile-local).

    bonds_ccl: read both spin planes (8) + write the label (2) + the two link
               bit planes (0.25) + the tile's edge slots and edge-link masks
               ((2 (64 + rows) + 16) / (64 rows))
    flip:      read the label (2), read and write both spin planes (16), write
               the tile's edge copies and read the neighbours' ((64 + rows) 16
               / (64 rows))
    fused:     flip of sweep t plus links / labels of sweep t+1 from the same
               spins: the flip's bytes + the label, planes and edge records of
               sweep t+1
    merge, finalize: only tile-edge records / per-tile sums: not counted
    """
    sites = 64.0 * tile_rows
    edge_rec = (2.0 * (64 + tile_rows) + 16.0) / sites
    edge_copies = (64 + tile_rows) * 16.0 / sites
    bonds = 8.0 + 2.0 + 0.25 + edge_rec
    flip = 2.0 + 16.0 + edge_copies
    if kernel == "bonds_ccl":
        return bonds
    if kernel == "flip":
        return flip
    if kernel == "fused":
        return flip + 2.0 + 0.25 + edge_rec
    return 0.0


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_from_counters(kernel: str, launches_sites: int):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter runs,
    or None when they are missing or were taken on a different kernel source."""
    try:
        rec = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return (k["fetch_kib"] + k["write_kib"]) * 1024.0 * rec.get("copy_scale", 1.0)


def valu_from_counters(kernel: str):
    """SQ_INSTS_VALU (wave instructions, all waves) per launch of `kernel` from
    the committed rocprofv3 counter run, or None when missing or stale."""
    try:
        rec = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return rec.get("kernels", {}).get(kernel, {}).get("valu_insts")


def cpu_baseline(L: int, beta: float, seed: int, nsweeps: int, state):
    """The oracle on this host's CPU, one thread, continuing the GPU's thermalised
    lattice (state = (cos, sin, sweeps done)) for nsweeps sweeps."""
    import numpy as np

    import oracle

    c, s, t = state
    lat = oracle.Lattice(L=L, beta=beta, seed=seed, storage32=True, t=int(t), c=c.astype(np.float64),
                         s=s.astype(np.float64))
    t0 = time.perf_counter()
    lat.run(nsweeps)
    dt = time.perf_counter() - t0
    return {"value": nsweeps * L * L / dt, "unit": "spin updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d sweeps (sweeps %d..%d) of the L=%d, beta=%g lattice continued from the GPU's "
                      "thermalised state, 1 thread (FP64, BFS labelling), %.1f s" % (nsweeps, t, t + nsweeps - 1,
                                                                                     L, beta, dt),
            "host_cpus": os.cpu_count()}


def copy_bandwidth(mib: int = 1024) -> float:
    """GB/s of a plain device-to-device copy of mib MiB (read + write bytes
    over the copy's time, HIP events), the achievable HBM figure of this box."""
    import torch

    src = torch.ones(mib * 2 ** 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * mib * 2 ** 20 / (ms * 1e-3) / 1e9


def cpu_batched(specs, nsweeps: int):
    """The oracle over every replica of the batch: one replica per task on a pool
    of host threads (the C oracle runs outside the GIL), nsweeps sweeps each from
    the oracle's own hot starts (the starts are inside the timed region)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))

    def one(sp):
        lat = oracle.Lattice(L=sp["L"], beta=sp["beta"], seed=sp["seed"], rep=sp["rep"], storage32=True)
        lat.run(nsweeps)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, sorted(specs, key=lambda sp: -sp["L"])))  # largest first
    dt = time.perf_counter() - t0
    total = sum(sp["L"] ** 2 for sp in specs)
    return {"value": nsweeps * total / dt, "unit": "spin updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d sweeps of all %d replicas of the batch (hot starts included), %d threads, %.1f s"
                      % (nsweeps, len(specs), threads, dt)}


def bench_l65536(sweeps: int):
    """Generalized-PCC run of one L = 65536 lattice (64-bit labels), beta0 = 1.0,
    window 1, dbeta 0.004 halved every 250 steps down to 0.0005."""
    import torch
    import paper_1210_6116_amd as xy
    import xyworkloads as wl

    from paper_1210_6116_amd import autotune

    L = 65536
    spec = dict(L=L, beta=1.0, seed=wl.SEED_L65536, label_bits=64)

    def pcc_step(h, n):
        h.pcc(n, 1, 0.004, dbeta_min=0.0005, halve_every=250)

    # merge schedule for this workload, timed by the autotuner on its own PCC
    # call (a short budget: blocks of a few sweeps of 2^32 sites separate the
    # choices)
    t0 = time.perf_counter()
    merge, merge_ms = autotune.tune_merge([spec], 32, sweeps=6, warmup=20, repeats=2, step=pcc_step, tag="pcc-w1")
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    lat = xy.Lattices(spec, stream=stream)
    autotune.configure(lat, merge)
    torch.cuda.synchronize()
    t_alloc = time.perf_counter() - t0
    lat.pcc(2, 1, 0.004, dbeta_min=0.0005, halve_every=250)  # warm-up steps
    torch.cuda.synchronize()
    lat.timing(True)
    t0 = time.perf_counter()
    means = lat.pcc(sweeps, 1, 0.004, dbeta_min=0.0005, halve_every=250, means=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    every = max(1, sweeps // 40)
    beta_trace = [float(b) for b in means["beta"][every - 1::every, 0]]
    ms, n, per = lat.timing_read(sweeps)
    lat.timing(False)
    beta = lat.beta()
    arena_gb = lat.bytes / 1e9
    lat.close()
    del lat
    torch.cuda.empty_cache()
    per = list(per)
    return {"workload": "PCC run, L=65536, uint64 canonical labels, beta0=1.0, window 1, dbeta 0.004 halved every "
                        "250 steps (floor 0.0005); %d timed sweeps after 2" % sweeps,
            "value": sweeps * L * L / dt, "unit": "spin updates/s", "ms_per_sweep": dt / sweeps * 1e3,
            "sweep_ms_p50": percentile(per, 50), "sweep_ms_p99": percentile(per, 99),
            "kernels_ms": {k: ms[i] / n[i] for i, k in enumerate(xy._lib.KERNEL_NAMES) if n[i] and k != "sweep"},
            "beta_after": beta, "beta_trace_every": every, "beta_trace": beta_trace,
            "arena_GB": arena_gb, "alloc_init_s": t_alloc,
            "merge_schedule": {"dedup": merge[0], "edges_per_wave": merge[1], "in_pass": merge[2],
                               "tuned_ms_per_sweep": {"%d,%d,%d" % k: v * 1e3 for k, v in merge_ms.items()},
                               "tune_s": t_tune}}


def bench_batched(sweeps: int, nrep: int = 512):
    """512 replicas of log-uniform L in 64..2048 and beta in [1.0, 1.2]: all in
    one handle (one launch per kernel per sweep, replayed from a HIP graph)
    against the same replicas swept one after another through plain handles."""
    import torch
    import paper_1210_6116_amd as xy
    import xyworkloads as wl

    from paper_1210_6116_amd import autotune

    specs = wl.batched_replicas(nrep)
    total = sum(sp["L"] ** 2 for sp in specs)
    # tile height picked by the autotuner for this replica set (timed here, not cached)
    rows, tune_s = autotune.tune(specs, use_cache=False)
    merge, merge_s = autotune.tune_merge(specs, rows, use_cache=False)
    specs = [dict(sp, tile_rows=rows) for sp in specs]
    chunk = 10 if sweeps % 10 == 0 else 1
    stream = torch.cuda.Stream()
    bat = xy.Lattices(specs, stream=stream)
    autotune.configure(bat, merge)
    bat.sweep_graph(chunk, 1)  # capture + warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bat.sweep_graph(chunk, sweeps // chunk)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    # latency of one round (one replay of the graph: `chunk` sweeps of every
    # replica), from events on the handle's stream
    rounds = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        bat.sweep_graph(chunk, 1)
        e1.record(stream)
        e1.synchronize()
        rounds.append(e0.elapsed_time(e1))
    bat.close()
    del bat
    plain = [xy.Lattices(sp, stream=stream) for sp in specs]
    for lat in plain:
        autotune.configure(lat, merge)
    for lat in plain:
        lat.sweep(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in plain:
        lat.sweep(sweeps)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    for lat in plain:
        lat.close()
    del plain
    torch.cuda.empty_cache()
    return {"workload": "%d replicas, L log-uniform over 64..2048, beta uniform on [1.0, 1.2], %d timed sweeps "
                        "each; batched = one handle replayed from a %d-sweep HIP graph; plain = one handle per "
                        "replica, swept one after another; both with the autotuned tile height" % (nrep, sweeps, chunk),
            "tile_rows": rows, "autotune_ms_per_sweep": {str(k): v * 1e3 for k, v in sorted(tune_s.items())},
            "merge_schedule": {"dedup": merge[0], "edges_per_wave": merge[1], "in_pass": merge[2],
                               "ms_per_sweep": {"%d,%d,%d" % k: v * 1e3 for k, v in sorted(merge_s.items())}},
            "round_sweeps": chunk, "round_ms_p50": percentile(rounds, 50), "round_ms_p99": percentile(rounds, 99),
            "spins": total, "batched_value": sweeps * total / dt_b, "plain_value": sweeps * total / dt_p,
            "unit": "spin updates/s", "speedup": dt_p / dt_b}


def bench_serving(n_requests: int, sweeps_lo: int, sweeps_hi: int, sequential: bool = True, deadline=None):
    """Poisson (20/s) stream of PCC run requests, L = 256..8192, admitted by a
    200 GB HBM budget and 64 slots, served by continuous batching; then the same
    trace one request at a time on plain handles (same PCC rule, same random
    streams, so every request ends with the same beta bit for bit)."""
    import xyworkloads as wl
    from paper_1210_6116_amd.serve import serve, serve_sequential

    trace = wl.serving_trace(n_requests=n_requests, sweeps_lo=sweeps_lo, sweeps_hi=sweeps_hi)
    last = [0.0]

    def progress_for(what):
        def progress(done, total, t):
            if t - last[0] >= 20.0 or done == total:
                last[0] = t
                print("bench: %s %d/%d requests done at %.0f s" % (what, done, total, t), file=sys.stderr,
                      flush=True)
        return progress

    res = serve(trace, budget_bytes=200 * 10 ** 9, max_slots=64, round_sweeps=16, progress=progress_for("served"))
    s = res["summary"]
    offered = s["offered_updates"] / (max(r["arrival"] for r in trace) + 1e-9)
    out = {"workload": "%d requests, Poisson rate 20/s, L = 2^(8..13), %d-%d sweeps each, PCC window 1 (dbeta 0.004 "
                       "halved every 250 steps, floor 0.0005), 200 GB budget, 64 slots, FIFO admission"
                       % (n_requests, sweeps_lo, sweeps_hi),
           "served_value": s["served_updates_per_s"], "unit": "spin updates/s",
           "ttc_p50_s": s["ttc_p50_s"], "ttc_p99_s": s["ttc_p99_s"], "makespan_s": s["makespan_s"],
           "mean_running": s["mean_running"], "offered_updates_per_s": offered}
    if sequential:
        last[0] = 0.0
        seq = serve_sequential(trace, progress=progress_for("sequential plain"), deadline=deadline)
        q = seq["summary"]
        served_by_id = {(r["seed"], r["arrival"]): r for r in res["requests"]}
        same = all(served_by_id[(b["seed"], b["arrival"])]["beta"] == b["beta"] for b in seq["requests"])
        out["sequential_plain"] = {"value": q["served_updates_per_s"], "ttc_p50_s": q["ttc_p50_s"],
                                   "ttc_p99_s": q["ttc_p99_s"], "makespan_s": q["makespan_s"],
                                   "requests": q["n"], "complete": q["complete"],
                                   "what": "the same trace, one request at a time in arrival order, each on its own "
                                           "plain handle" + ("" if q["complete"] else
                                                             "; stopped at the bench's time budget after the first "
                                                             "%d requests (rate over those)" % q["n"])}
        out["served_over_sequential"] = s["served_updates_per_s"] / q["served_updates_per_s"]
        out["final_beta_identical"] = same
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed sweeps after the %d thermalisation sweeps" % THERM_SWEEPS)
    ap.add_argument("--L", type=int, default=4096)
    ap.add_argument("--beta", type=float, default=1.12)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--merge-schedule", default="",
                    help="'dedup,edges_per_wave[,in_pass]' for the L = 4096 lattice instead of the autotuner's pick "
                         "(counter runs, whose slowed kernels can rank the choices differently)")
    ap.add_argument("--cpu-sweeps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle's CPU baseline")
    ap.add_argument("--no-instrument", action="store_true", help="skip the instrumented pass")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the L=65536 PCC, batched and serving legs")
    ap.add_argument("--extras", default="l65536,batched,serving",
                    help="comma-separated subset of the extra workloads to run")
    ap.add_argument("--l65536-sweeps", type=int, default=2000)
    ap.add_argument("--batched-sweeps", type=int, default=1000)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-sweeps-lo", type=int, default=1000)
    ap.add_argument("--serve-sweeps-hi", type=int, default=10000)
    ap.add_argument("--no-serve-sequential", action="store_true",
                    help="skip the one-request-at-a-time plain leg of the serving trace")
    ap.add_argument("--time-budget", type=float, default=520.0,
                    help="seconds of bench wall time after which no further extra leg starts (the serving "
                         "trace's sequential leg stops starting requests); the headline line always prints")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run a plain elementwise copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the sweep runs on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1210_6116_amd as xy
    import xyworkloads as wl

    t_start = time.perf_counter()
    if args.copy_calib_mb:
        src = torch.ones(args.copy_calib_mb * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    L, beta = args.L, args.beta
    N = L * L
    seed = wl.SEED_L4096
    print("bench: L=%d beta=%g thermalisation=%d warmup=%d steps=%d" % (L, beta, THERM_SWEEPS, args.warmup,
                                                                      args.steps), file=sys.stderr, flush=True)
    from paper_1210_6116_amd import autotune

    rows = args.tile_rows or 32
    # merge schedule picked by the autotuner for this lattice (timed here, not cached)
    if args.merge_schedule:
        merge, merge_s = tuple(int(x) for x in (args.merge_schedule + ",0").split(",")[:3]), {}
    else:
        merge, merge_s = autotune.tune_merge([dict(L=L, beta=beta, seed=seed)], rows, use_cache=False)
    stream = torch.cuda.Stream()
    lat = xy.Lattices(dict(L=L, beta=beta, seed=seed, tile_rows=rows), stream=stream)
    autotune.configure(lat, merge)
    label_bits = 64 if N >= 2 ** 32 else 32

    lat.sweep(THERM_SWEEPS)
    lat.sweep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps * N / dt
    print("bench: timed %d sweeps in %.3f s" % (args.steps, dt), file=sys.stderr, flush=True)

    bps = SWEEP_BYTES[label_bits]
    roofline = None
    valu_issue = None
    latency = {}
    kernels = {}
    if not args.no_instrument:
        # same call shape as the timed pass (one call of --steps sweeps), with
        # HIP events around every kernel and every sweep on the handle's stream
        lat.timing(True)
        lat.sweep(args.steps)
        ms, launches, per_sweep = lat.timing_read(args.steps)
        lat.timing(False)
        per_sweep = list(per_sweep)
        latency = {"sweep_ms_p50": percentile(per_sweep, 50), "sweep_ms_p99": percentile(per_sweep, 99),
                   "sweep_ms_mean": sum(per_sweep) / len(per_sweep)}
        for k, name in enumerate(xy._lib.KERNEL_NAMES):
            if launches[k] and name != "sweep":
                avg = ms[k] / launches[k]
                ab = alg_bytes_per_site(name, rows) * N
                kernels[name] = {"launches": int(launches[k]), "avg_ms": avg, "design_bytes": ab,
                                 "design_GBps": (ab / (avg * 1e-3) / 1e9) if ab else None}
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
        kd = kernels[dom]
        # the dominant kernel completes one sweep of every site per launch (the
        # flip of one sweep and the links and labels of the next): its
        # algorithmic bytes are the sweep's 24 B (32-bit labels) per site
        alg = bps * N if dom == "fused" else kd["design_bytes"]
        achieved = alg / (kd["avg_ms"] * 1e-3) / 1e9
        copy_gbs = copy_bandwidth()
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_counters(dom, N),
                    "alg_bytes_per_site": bps if dom == "fused" else alg / N, "alg_bytes_per_launch": alg,
                    "avg_launch_ms": kd["avg_ms"], "launches": kd["launches"],
                    # the kernel's own byte model (16-bit tile-local labels, edge records)
                    "design_bytes_per_site": kd["design_bytes"] / N,
                    "design_frac": kd["design_GBps"] / HBM_PEAK_GBS if kd["design_GBps"] else None,
                    # the whole sweep (every kernel and launch gap) against the same roofline
                    "sweep_achieved": value * bps / 1e9, "sweep_frac": value * bps / 1e9 / HBM_PEAK_GBS,
                    "copy_GBps": copy_gbs, "copy_frac": copy_gbs / HBM_PEAK_GBS}
        vi = valu_from_counters(dom)
        if vi:
            # the same kernel against its instruction-issue ceiling
            rate = vi * 64 / (kd["avg_ms"] * 1e-3) / 1e12
            valu_issue = {"bound": "alu", "kernel": dom, "achieved": rate, "peak": VALU_PEAK_TLANE,
                          "unit": "T VALU lane-instructions/s", "frac": rate / VALU_PEAK_TLANE,
                          "valu_insts_per_launch": vi}
    # the thermalised lattice the CPU oracle continues from (taken after the
    # timed sweeps, so that no host copy idles the GPU before them)
    therm_state = (*lat.get_state(), lat.sweep_count()[0]) if not args.no_cpu else None
    lat.close()
    del lat
    torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(L, beta, seed, args.cpu_sweeps, therm_state)

    line = {
        "metric": "spin updates/sec (SW sweeps x L^2 / s)",
        "value": value,
        "unit": "spin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the paper's only single-GPU timing (L = 4096, 500,000 MCS with measurements in
        # about 14 h on one GeForce GTX580): another machine, quoted as context
        "paper_context": {"value": 4096 ** 2 * 5e5 / (14 * 3600.0), "unit": "spin updates/s",
                          "hardware": "1 x GeForce GTX580", "ratio": value / (4096 ** 2 * 5e5 / (14 * 3600.0))},
        "dtype": "f32 state, f64 reflection and sums",
        "data": "synthetic (seeded Philox hot start)",
        "config": {"workload": "plain SW sweep, 2D XY periodic L=%d, beta=%g, uint%d canonical labels "
                               "(16-bit tile-local labels in the sweep), hot start, %d thermalisation + %d "
                               "warm-up sweeps untimed, %d timed sweeps" % (L, beta, label_bits, THERM_SWEEPS,
                                                                            args.warmup, args.steps),
                   "L": L, "beta": beta, "seed": seed, "thermalisation": THERM_SWEEPS,
                   "merge_schedule": {"dedup": merge[0], "edges_per_wave": merge[1], "in_pass": merge[2],
                                      "tuned_ms_per_sweep": {"%d,%d,%d" % k: v * 1e3
                                                             for k, v in sorted(merge_s.items())}},
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "valu_issue": valu_issue,
        "latency": latency,
        "kernels": kernels,
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    if not args.no_extras:
        extras = {}
        chosen = set(args.extras.split(","))
        deadline = t_start + args.time_budget
        # rough wall time of each leg at MI355X speed (seconds), to skip a leg
        # that would run past the budget rather than be cut off by a caller
        est = {"l65536": 16.0 + 0.04 * args.l65536_sweeps, "batched": 12.0 + 0.025 * args.batched_sweeps,
               # the served pass: requests x mean L^2 (1.49e7 for L = 256..8192) x mean sweeps at ~1e11 updates/s
               # (the sequential pass after it stops starting requests at the deadline)
               "serving": 10.0 + args.serve_requests * 1.49e7 * (args.serve_sweeps_lo + args.serve_sweeps_hi) / 2.0
               / 1.0e11}
        for key, name, fn in (("l65536", "L65536_pcc", lambda: bench_l65536(args.l65536_sweeps)),
                              ("batched", "batched_vs_plain", lambda: bench_batched(args.batched_sweeps)),
                              ("serving", "serving", lambda: bench_serving(args.serve_requests, args.serve_sweeps_lo,
                                                                           args.serve_sweeps_hi,
                                                                           not args.no_serve_sequential,
                                                                           deadline=deadline))):
            if key not in chosen:
                continue
            now = time.perf_counter()
            if now + est[key] > deadline:
                extras[name] = {"skipped": "time budget: %.0f s left of --time-budget %.0f, the leg takes about %.0f s"
                                           % (deadline - now, args.time_budget, est[key])}
                continue
            print("bench: %s (at %.0f s)" % (name, now - t_start), file=sys.stderr, flush=True)
            try:
                extras[name] = fn()
            except Exception as exc:  # reported, not hidden: the headline line still prints
                extras[name] = {"error": "%s: %s" % (type(exc).__name__, exc)}
            print("bench: %s done (at %.0f s)" % (name, time.perf_counter() - t_start), file=sys.stderr, flush=True)
            if key == "batched" and not args.no_cpu and "error" not in extras[name]:
                extras[name]["cpu_baseline"] = cpu_batched(wl.batched_replicas(512), 1)
        line["extras"] = extras
    line["bench_wall_s"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
