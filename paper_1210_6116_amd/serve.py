"""Serving loop: continuous batching of PCC run requests on one GPU.

Requests (one lattice each: L, seed, initial beta, number of sweeps) arrive over
time.  They are admitted in arrival order into a native group (xy_group_* in
libxy.so) as soon as a slot and enough of the group's HBM budget are free; all
admitted requests are swept together, round by round, in the same kernel
launches, each with its own generalized-PCC beta updates; a finished request
frees its slot and memory for the next.  Reported: time to completion (TTC) of
every request from its arrival, p50 / p99 TTC, and served spin updates per
second over the makespan.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib
from ._lib import XY_START_HOT, xy_params, xy_pcc

PCC_TARGET = 0.636508


def request_bytes(L: int) -> int:
    """Bytes one request of side L occupies in a group's budget (host-side arithmetic)."""
    return _lib.xy_group_bytes(xy_params(L=L, beta=1.0, seed=0, replica=0, label_bits=0, start=XY_START_HOT,
                                         tile_rows=0))


class Group:
    """A native serving group on a torch stream."""

    def __init__(self, budget_bytes: int, max_slots: int, pcc: xy_pcc, stream: torch.cuda.Stream | None = None):
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.g = _lib.xy_group_create(int(budget_bytes), int(max_slots), pcc, self.stream.cuda_stream)

    def add(self, L: int, seed: int, beta0: float, sweeps: int, replica: int = 0):
        p = xy_params(L=L, beta=beta0, seed=seed & (2 ** 64 - 1), replica=replica, label_bits=0,
                      start=XY_START_HOT, tile_rows=0)
        return _lib.xy_group_add(self.g, p, sweeps)

    def round(self, max_sweeps: int) -> int:
        return _lib.xy_group_round(self.g, max_sweeps)

    def poll(self):
        return _lib.xy_group_poll(self.g)

    def result(self, slot: int):
        return _lib.xy_group_result(self.g, slot)

    def get_state(self, slot: int, L: int):
        """(cos, sin) float32 arrays of the request in `slot` (side L)."""
        c = np.zeros(L * L, dtype=np.float32)
        s = np.zeros(L * L, dtype=np.float32)
        _lib.xy_group_get_state(self.g, slot, c, s)
        return c, s

    def release(self, slot: int):
        _lib.xy_group_release(self.g, slot)

    def info(self):
        return _lib.xy_group_info(self.g)

    def close(self):
        if getattr(self, "g", None) is not None:
            _lib.xy_group_free(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(trace, budget_bytes: int = 200 * 10 ** 9, max_slots: int = 64, pcc: xy_pcc | None = None,
          round_sweeps: int = 16, clock=time.perf_counter, sleep=time.sleep, progress=None):
    """Runs the request trace in real time (arrival times in seconds from start).

    trace: list of dicts with arrival, L, sweeps, seed, beta0.  Returns a dict
    with per-request records and the summary (makespan, served updates/s,
    p50 / p99 TTC in seconds, mean slots in use).  progress, if given, is
    called as progress(finished, total, seconds) whenever requests finish.
    """
    if pcc is None:
        pcc = xy_pcc(window=1, dbeta0=0.004, dbeta_min=0.0005, halve_every=250, target=PCC_TARGET)
    # a request larger than the whole budget could never be admitted, and FIFO
    # admission would then wait for it for ever: refuse the trace up front
    for k, r in enumerate(trace):
        need = request_bytes(r["L"])
        if need > budget_bytes:
            raise ValueError("request %d (L=%d) needs %d bytes, more than the %d-byte budget"
                             % (k, r["L"], need, budget_bytes))
    order = sorted(range(len(trace)), key=lambda k: trace[k]["arrival"])
    grp = Group(budget_bytes, max_slots, pcc)
    recs = {k: dict(trace[k]) for k in order}
    slot_of = {}
    nxt = 0
    t0 = clock()
    running_samples = []
    finished = 0
    while nxt < len(order) or slot_of:
        now = clock() - t0
        # admit in arrival order while the head fits
        while nxt < len(order) and recs[order[nxt]]["arrival"] <= now:
            k = order[nxt]
            r = recs[k]
            slot = grp.add(r["L"], r["seed"], r["beta0"], r["sweeps"], replica=k)
            if slot is None:
                break
            r["admitted"] = now
            slot_of[slot] = k
            nxt += 1
        if not slot_of:
            if nxt < len(order):
                sleep(max(0.0, recs[order[nxt]]["arrival"] - (clock() - t0)))
            continue
        running_samples.append(len(slot_of))
        grp.round(round_sweeps)
        done_t = clock() - t0
        polled = grp.poll()
        for slot in polled:
            k = slot_of.pop(slot)
            last, beta, beta_mean = grp.result(slot)
            recs[k].update(finished=done_t, ttc=done_t - recs[k]["arrival"], beta=beta, beta_mean=beta_mean,
                           E=float(last["E"]), m2=float(last["m2"]))
            grp.release(slot)
        finished += len(polled)
        if polled and progress is not None:
            progress(finished, len(order), done_t)
    grp.close()
    makespan = max(r["finished"] for r in recs.values()) - min(r["arrival"] for r in recs.values())
    updates = sum(r["L"] * r["L"] * r["sweeps"] for r in recs.values())
    ttc = np.array([r["ttc"] for r in recs.values()])
    return dict(requests=[recs[k] for k in sorted(recs)],
                summary=dict(n=len(recs), makespan_s=makespan, served_updates_per_s=updates / makespan,
                             ttc_p50_s=float(np.percentile(ttc, 50)), ttc_p99_s=float(np.percentile(ttc, 99)),
                             mean_running=float(np.mean(running_samples)) if running_samples else 0.0,
                             offered_updates=updates))


def serve_sequential(trace, pcc: xy_pcc | None = None, clock=time.perf_counter, sleep=time.sleep, progress=None,
                     deadline: float | None = None):
    """The same trace without batching: one request at a time in arrival order,
    each on its own plain handle (one lattice, the same PCC rule), started when
    it has arrived and the previous one has finished.  Same records and summary
    as serve().  deadline (a clock() value): no request is started after it;
    the summary then covers the requests that ran (complete = False)."""
    from . import Lattices

    if pcc is None:
        pcc = xy_pcc(window=1, dbeta0=0.004, dbeta_min=0.0005, halve_every=250, target=PCC_TARGET)
    order = sorted(range(len(trace)), key=lambda k: trace[k]["arrival"])
    recs = {k: dict(trace[k]) for k in order}
    stream = torch.cuda.Stream()
    t0 = clock()
    ran = []
    for done, k in enumerate(order):
        if deadline is not None and clock() > deadline:
            break
        r = recs[k]
        ran.append(k)
        wait = r["arrival"] - (clock() - t0)
        if wait > 0:
            sleep(wait)
        r["admitted"] = clock() - t0
        lat = Lattices(dict(L=r["L"], beta=r["beta0"], seed=r["seed"], rep=k), stream=stream)
        lat.pcc(r["sweeps"], pcc.window, pcc.dbeta0, dbeta_min=pcc.dbeta_min, halve_every=pcc.halve_every,
                target=pcc.target)
        beta = lat.beta()  # synchronizes the stream
        last = lat.measure()[0]
        lat.close()
        done_t = clock() - t0
        r.update(finished=done_t, ttc=done_t - r["arrival"], beta=beta, E=float(last["E"]), m2=float(last["m2"]))
        if progress is not None:
            progress(done + 1, len(order), done_t)
    done_recs = [recs[k] for k in ran]
    makespan = max(r["finished"] for r in done_recs) - min(r["arrival"] for r in done_recs)
    updates = sum(r["L"] * r["L"] * r["sweeps"] for r in done_recs)
    ttc = np.array([r["ttc"] for r in done_recs])
    return dict(requests=[recs[k] for k in sorted(ran)],
                summary=dict(n=len(done_recs), complete=len(done_recs) == len(order), makespan_s=makespan,
                             served_updates_per_s=updates / makespan,
                             ttc_p50_s=float(np.percentile(ttc, 50)), ttc_p99_s=float(np.percentile(ttc, 99)),
                             mean_running=1.0, offered_updates=updates))
