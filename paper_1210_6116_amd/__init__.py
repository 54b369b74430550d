"""MI355X-native Swendsen-Wang / PCC engine for the 2D classical XY model.

Implements the hot path of Komura & Okabe, "Large-scale Monte Carlo simulation
of two-dimensional classical XY model using multiple GPUs" (arXiv:1210.6116):
the Swendsen-Wang multi-cluster update with Wolff's embedded-cluster formalism
on a periodic L x L lattice (Eq. (Hc)), the energy / magnetisation / helicity
modulus reductions, and the generalized probability-changing-cluster (PCC)
controller that moves beta towards beta*Upsilon = 0.636508.

The work runs in hand-written HIP kernels for gfx950 inside libxy.so (C ABI:
include/xy.h).  This package is a thin binding: ``_lib`` mirrors the C calls
one to one, and ``Lattices`` keeps a handle together with the torch tensor
that holds its device memory and the torch stream it runs on.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import (OBS_DTYPE, XY_PCC_HELICITY, XY_PCC_PERCOLATION, XY_START_COLD, XY_START_HOT, XYError, xy_obs,
                   xy_params, xy_pcc)

__all__ = ["Lattices", "XYError", "OBS_DTYPE", "XY_START_HOT", "XY_START_COLD", "PCC_TARGET",
           "unpack_bits", "xy_params", "xy_obs", "xy_pcc", "XY_PCC_HELICITY", "XY_PCC_PERCOLATION"]

PCC_TARGET = 0.636508  # critical beta*Upsilon with the periodic-boundary winding correction


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """Bit i of word i/32 (little-endian) -> uint8 array of n values."""
    return np.unpackbits(np.ascontiguousarray(words, dtype="<u4").view(np.uint8), bitorder="little")[:n]


def _params(spec: dict) -> xy_params:
    return xy_params(L=int(spec["L"]), beta=float(spec["beta"]), seed=int(spec["seed"]) & (2 ** 64 - 1),
                     replica=int(spec.get("rep", spec.get("replica", 0))),
                     label_bits=int(spec.get("label_bits", 0)),
                     start=int(spec.get("start", XY_START_HOT)), tile_rows=int(spec.get("tile_rows", 0)))


class Lattices:
    """A set of replicas (each its own L, beta, seed, stream id) updated together.

    Device memory is one torch uint8 tensor (the arena); work is enqueued on a
    torch stream (the current one unless given).
    """

    def __init__(self, replicas, stream: torch.cuda.Stream | None = None, device: str = "cuda"):
        if isinstance(replicas, dict):
            replicas = [replicas]
        self.specs = [dict(r) for r in replicas]
        self.params = [_params(r) for r in self.specs]
        self.n = len(self.params)
        self.L = [p.L for p in self.params]
        self.N = [p.L * p.L for p in self.params]
        self.bytes = _lib.xy_bytes_required(self.params)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.arena = torch.empty(self.bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)  # the arena's memory is free of earlier torch work
        self.h = _lib.xy_alloc(self.params, self.stream.cuda_stream, self.arena.data_ptr(), self.bytes)

    # ---------------------------------------------------------------- sweeps
    def sweep(self, nsweeps: int, trace: bool = False):
        """nsweeps sweeps; with trace=True returns observables [nsweeps, n] (OBS_DTYPE)."""
        out = np.zeros((nsweeps, self.n), dtype=OBS_DTYPE) if trace else None
        _lib.xy_sweep(self.h, nsweeps, out)
        return out

    def sweep_graph(self, nsweeps: int, replays: int):
        """replays x nsweeps sweeps from one captured HIP graph of nsweeps sweeps."""
        _lib.xy_sweep_graph(self.h, nsweeps, replays)

    def measure(self):
        out = np.zeros(self.n, dtype=OBS_DTYPE)
        _lib.xy_measure(self.h, out)
        return out

    def pcc(self, nsteps: int, window: int, dbeta0: float, dbeta_min: float = 0.0, halve_every: int = 0,
            target: float = PCC_TARGET, means: bool = False, rule: int = XY_PCC_HELICITY):
        """nsteps PCC steps of `window` sweeps; with means=True returns window means [nsteps, n].
        rule: XY_PCC_HELICITY (the paper's rule, target 0.636508) or XY_PCC_PERCOLATION
        (the original rule on whether the clusters wind around the lattice, target e.g. 0.5)."""
        c = xy_pcc(window=window, dbeta0=dbeta0, dbeta_min=dbeta_min, halve_every=halve_every, target=target,
                   rule=rule)
        out = np.zeros((nsteps, self.n), dtype=OBS_DTYPE) if means else None
        _lib.xy_pcc_step(self.h, c, nsteps, out)
        return out

    # ------------------------------------------------------------ inspection
    def get_state(self, rep: int = 0):
        c = np.zeros(self.N[rep], dtype=np.float32)
        s = np.zeros(self.N[rep], dtype=np.float32)
        _lib.xy_get_state(self.h, rep, c, s)
        return c, s

    def set_state(self, c, s, rep: int = 0):
        _lib.xy_set_state(self.h, rep, np.ascontiguousarray(c, dtype=np.float32),
                          np.ascontiguousarray(s, dtype=np.float32))

    def labels(self, rep: int = 0) -> np.ndarray:
        out = np.zeros(self.N[rep], dtype=np.int64)
        _lib.xy_get_labels(self.h, rep, out)
        return out

    def bonds(self, rep: int = 0):
        """Active links of the latest sweep as uint8 per site (bx, by)."""
        words = max(1, (self.N[rep] + 31) // 32)
        bx = np.zeros(words, dtype=np.uint32)
        by = np.zeros(words, dtype=np.uint32)
        _lib.xy_get_bonds(self.h, rep, bx, by)
        return unpack_bits(bx, self.N[rep]), unpack_bits(by, self.N[rep])

    def views(self, rep: int = 0) -> dict:
        """Device tensors (no copies) of the state and link planes after the
        latest sweep: cos, sin (float32, N), bx, by (int32 words).  Valid until
        the next call on the handle."""
        v = _lib.xy_get_views(self.h, rep)
        base = self.arena.data_ptr()
        N = self.N[rep]
        words = max(1, (N + 31) // 32)

        def sub(ptr, nbytes, dtype):
            off = ptr - base
            assert 0 <= off and off + nbytes <= self.bytes
            return self.arena[off:off + nbytes].view(dtype)

        return {"cos": sub(v.cos_plane, 4 * N, torch.float32), "sin": sub(v.sin_plane, 4 * N, torch.float32),
                "bx": sub(v.bond_x, 4 * words, torch.int32), "by": sub(v.bond_y, 4 * words, torch.int32),
                "label_bits": v.label_bits, "L": v.L, "sweep": v.sweep}

    def labels_device(self, rep: int = 0, bits: int = 64) -> torch.Tensor:
        """Canonical labels of the latest sweep in a new device tensor (int64,
        or int32 holding the unsigned 32-bit labels)."""
        out = torch.empty(self.N[rep], dtype=torch.int64 if bits == 64 else torch.int32, device=self.device)
        _lib.xy_flatten_labels(self.h, rep, out.data_ptr(), bits)
        return out

    def beta(self, rep: int = 0) -> float:
        return _lib.xy_get_beta(self.h, rep)

    def set_beta(self, beta: float, rep: int = 0):
        _lib.xy_set_beta(self.h, rep, beta)

    def sweep_count(self, rep: int = 0):
        """(sweeps completed, mirror direction of the next sweep)."""
        return _lib.xy_get_sweep(self.h, rep)

    def set_merge(self, dedup: int, edges_per_wave: int = 1):
        """Merge schedule: pair deduplication (_lib.XY_DEDUP_WAVE, XY_DEDUP_NEIGHBOUR or
        XY_DEDUP_HASH) and tile edges per wave (1, 2 or 4)."""
        _lib.xy_set_merge(self.h, dedup, edges_per_wave)

    def set_merge_in_pass(self, on: bool):
        """Unite the tile edges inside the labelling tile pass (no merge kernel)."""
        _lib.xy_set_merge_in_pass(self.h, 1 if on else 0)

    def timing(self, enable: bool):
        _lib.xy_timing(self.h, enable)

    def timing_read(self, max_samples: int = 0):
        """(ms per kernel class, launches per class, per-sweep durations in ms)."""
        return _lib.xy_timing_read(self.h, max_samples)

    def close(self):
        if getattr(self, "h", None) is not None:
            _lib.xy_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def label_links(L: int, bx: np.ndarray, by: np.ndarray, label_bits: int = 32, tile_rows: int = 0,
                device: str = "cuda") -> np.ndarray:
    """Canonical labels of a given link set (uint8 per site) with the sweep's labelling kernels."""
    N = L * L
    words = max(1, (N + 31) // 32)

    def pack(b):
        bits = np.zeros(words * 32, dtype=np.uint8)
        bits[:N] = b
        return torch.from_numpy(np.packbits(bits, bitorder="little").view("<u4").astype(np.uint32).view(np.int32))

    dbx = pack(bx).to(device)
    dby = pack(by).to(device)
    lab = torch.empty(N, dtype=torch.int64 if label_bits == 64 else torch.int32, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    _lib.xy_label_links(L, label_bits, tile_rows, dbx.data_ptr(), dby.data_ptr(), lab.data_ptr(),
                        stream.cuda_stream)
    out = lab.cpu().numpy()
    return out.astype(np.int64) if label_bits == 64 else out.view(np.uint32).astype(np.int64)
