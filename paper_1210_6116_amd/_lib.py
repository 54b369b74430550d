"""ctypes binding of libxy.so (include/xy.h): argument marshalling only.

Every step of the sweep runs in the library's HIP kernels.  torch is imported
first so that the process holds a single HIP runtime (libxy.so and torch then
share it), and it supplies device memory (the arena tensor) and streams.
There is no fallback: if libxy.so is missing or fails to load, this raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime that libxy.so binds to)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libxy.so")

XY_OK, XY_EINVAL, XY_ENOMEM, XY_EDEVICE, XY_ESTATE, XY_EBUDGET = 0, -1, -2, -3, -4, -5
XY_START_HOT, XY_START_COLD = 0, 1
(XY_K_BONDS, XY_K_MERGE, XY_K_FLIP, XY_K_FUSED, XY_K_FINALIZE, XY_K_COINS, XY_K_SWEEP, XY_K_WRAP, XY_K_SPEC,
 XY_K_PLSEL, XY_K_COUNT) = range(11)
KERNEL_NAMES = ("bonds_ccl", "merge", "flip", "fused", "finalize", "coins", "sweep", "wrap", "flip_links2",
                "labels_chosen")
XY_PCC_HELICITY, XY_PCC_PERCOLATION = 0, 1
XY_DEDUP_WAVE, XY_DEDUP_NEIGHBOUR, XY_DEDUP_HASH = 0, 1, 2


class XYError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("xy error %d: %s" % (code, msg))
        self.code = code


class xy_params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int64), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica", ctypes.c_uint32), ("label_bits", ctypes.c_int32), ("start", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32)]


class xy_obs(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_uint64), ("beta", ctypes.c_double), ("E", ctypes.c_double),
                ("m2", ctypes.c_double), ("ex", ctypes.c_double), ("sx", ctypes.c_double),
                ("ey", ctypes.c_double), ("sy", ctypes.c_double), ("ups_x", ctypes.c_double),
                ("mk2", ctypes.c_double), ("near_ties", ctypes.c_uint64), ("wrap", ctypes.c_uint64),
                ("perc", ctypes.c_double)]


class xy_pcc(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int64), ("dbeta0", ctypes.c_double), ("dbeta_min", ctypes.c_double),
                ("halve_every", ctypes.c_int64), ("target", ctypes.c_double), ("rule", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class xy_views(ctypes.Structure):
    _fields_ = [("cos_plane", ctypes.c_void_p), ("sin_plane", ctypes.c_void_p),
                ("bond_x", ctypes.c_void_p), ("bond_y", ctypes.c_void_p), ("L", ctypes.c_int64),
                ("label_bits", ctypes.c_int32), ("reserved", ctypes.c_int32), ("sweep", ctypes.c_uint64)]


OBS_DTYPE = np.dtype([("sweep", np.uint64), ("beta", np.float64), ("E", np.float64), ("m2", np.float64),
                      ("ex", np.float64), ("sx", np.float64), ("ey", np.float64), ("sy", np.float64),
                      ("ups_x", np.float64), ("mk2", np.float64), ("near_ties", np.uint64), ("wrap", np.uint64),
                      ("perc", np.float64)])
assert OBS_DTYPE.itemsize == ctypes.sizeof(xy_obs)

_lib = None

# name -> (restype, argtypes); the C signatures of include/xy.h
_P = ctypes.POINTER
_SIGS = {
    "xy_bytes_required": (ctypes.c_int, [_P(xy_params), ctypes.c_int32, _P(ctypes.c_size_t)]),
    "xy_alloc": (ctypes.c_int, [_P(xy_params), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_size_t, _P(ctypes.c_void_p)]),
    "xy_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "xy_sweep_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]),
    "xy_measure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "xy_pcc_step": (ctypes.c_int, [ctypes.c_void_p, _P(xy_pcc), ctypes.c_int64, ctypes.c_void_p]),
    "xy_free": (ctypes.c_int, [ctypes.c_void_p]),
    "xy_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "xy_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "xy_get_labels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "xy_get_bonds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "xy_flatten_labels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]),
    "xy_get_views": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(xy_views)]),
    "xy_set_beta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double]),
    "xy_get_beta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_double)]),
    "xy_get_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_uint64), ctypes.c_void_p]),
    "xy_label_links": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "xy_label_links_noalloc": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "xy_set_merge": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "xy_set_merge_in_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "xy_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "xy_timing_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, _P(ctypes.c_int64)]),
    "xy_last_error": (ctypes.c_char_p, []),
    "xy_group_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, _P(xy_pcc), ctypes.c_void_p,
                                       _P(ctypes.c_void_p)]),
    "xy_group_add": (ctypes.c_int, [ctypes.c_void_p, _P(xy_params), ctypes.c_int64, _P(ctypes.c_int32)]),
    "xy_group_bytes": (ctypes.c_int, [_P(xy_params), _P(ctypes.c_size_t)]),
    "xy_group_round": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, _P(ctypes.c_int64)]),
    "xy_group_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_int32)]),
    "xy_group_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, _P(ctypes.c_double),
                                       _P(ctypes.c_double)]),
    "xy_group_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "xy_group_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "xy_group_info": (ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_size_t), _P(ctypes.c_int32)]),
    "xy_group_free": (ctypes.c_int, [ctypes.c_void_p]),
}
EXPORTS = tuple(_SIGS)


def load():
    """Loads libxy.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libxy.so is not built (%s); run paper_1210_6116_amd/build.py" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != XY_OK:
        raise XYError(rc, load().xy_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------- the C calls, same names
def xy_bytes_required(params) -> int:
    arr = (xy_params * len(params))(*params)
    out = ctypes.c_size_t(0)
    _check(load().xy_bytes_required(arr, len(params), ctypes.byref(out)))
    return out.value


def xy_alloc(params, stream=None, arena=None, arena_bytes=0):
    arr = (xy_params * len(params))(*params)
    h = ctypes.c_void_p()
    _check(load().xy_alloc(arr, len(params), stream, arena, arena_bytes, ctypes.byref(h)))
    return h


def xy_sweep(h, nsweeps: int, trace: np.ndarray | None = None):
    _check(load().xy_sweep(h, nsweeps, None if trace is None else _ptr(trace)))


def xy_sweep_graph(h, nsweeps: int, replays: int):
    _check(load().xy_sweep_graph(h, nsweeps, replays))


def xy_measure(h, out: np.ndarray):
    _check(load().xy_measure(h, _ptr(out)))


def xy_pcc_step(h, pcc: xy_pcc, nsteps: int, window_mean: np.ndarray | None = None):
    _check(load().xy_pcc_step(h, ctypes.byref(pcc), nsteps, None if window_mean is None else _ptr(window_mean)))


def xy_free(h):
    _check(load().xy_free(h))


def xy_get_state(h, rep: int, c: np.ndarray, s: np.ndarray):
    _check(load().xy_get_state(h, rep, _ptr(c), _ptr(s)))


def xy_set_state(h, rep: int, c: np.ndarray, s: np.ndarray):
    _check(load().xy_set_state(h, rep, _ptr(c), _ptr(s)))


def xy_get_labels(h, rep: int, out: np.ndarray):
    _check(load().xy_get_labels(h, rep, _ptr(out)))


def xy_get_bonds(h, rep: int, bx: np.ndarray, by: np.ndarray):
    _check(load().xy_get_bonds(h, rep, _ptr(bx), _ptr(by)))


def xy_flatten_labels(h, rep: int, d_out: int, out_bits: int):
    _check(load().xy_flatten_labels(h, rep, d_out, out_bits))


def xy_get_views(h, rep: int) -> xy_views:
    out = xy_views()
    _check(load().xy_get_views(h, rep, ctypes.byref(out)))
    return out


def xy_set_beta(h, rep: int, beta: float):
    _check(load().xy_set_beta(h, rep, beta))


def xy_get_beta(h, rep: int) -> float:
    b = ctypes.c_double(0.0)
    _check(load().xy_get_beta(h, rep, ctypes.byref(b)))
    return b.value


def xy_get_sweep(h, rep: int):
    t = ctypes.c_uint64(0)
    r = np.zeros(2)
    _check(load().xy_get_sweep(h, rep, ctypes.byref(t), _ptr(r)))
    return t.value, r


def xy_label_links(L: int, label_bits: int, tile_rows: int, d_bx: int, d_by: int, d_labels: int, stream=None):
    _check(load().xy_label_links(L, label_bits, tile_rows, d_bx, d_by, d_labels, stream))


def xy_label_links_noalloc(L: int, label_bits: int, tile_rows: int, d_bx: int, d_by: int, d_labels: int,
                           stream=None):
    _check(load().xy_label_links_noalloc(L, label_bits, tile_rows, d_bx, d_by, d_labels, stream))


def xy_set_merge(h, dedup: int, edges_per_wave: int):
    _check(load().xy_set_merge(h, int(dedup), int(edges_per_wave)))


def xy_set_merge_in_pass(h, on: int):
    _check(load().xy_set_merge_in_pass(h, int(on)))


def xy_timing(h, enable: bool):
    _check(load().xy_timing(h, int(enable)))


def xy_timing_read(h, max_samples: int = 0):
    """(ms[XY_K_COUNT], launches[XY_K_COUNT], per-sweep durations in ms)."""
    ms = np.zeros(XY_K_COUNT)
    n = np.zeros(XY_K_COUNT, dtype=np.int64)
    samples = np.zeros(max(1, max_samples))
    ns = ctypes.c_int64(0)
    _check(load().xy_timing_read(h, _ptr(ms), _ptr(n), _ptr(samples), max_samples, ctypes.byref(ns)))
    return ms, n, samples[:ns.value]


def xy_last_error() -> str:
    return load().xy_last_error().decode()


# ------------------------------------------------- serving group
def xy_group_create(budget_bytes: int, max_slots: int, pcc: xy_pcc, stream=None):
    g = ctypes.c_void_p()
    _check(load().xy_group_create(budget_bytes, max_slots, ctypes.byref(pcc), stream, ctypes.byref(g)))
    return g


def xy_group_bytes(params: xy_params) -> int:
    out = ctypes.c_size_t(0)
    _check(load().xy_group_bytes(ctypes.byref(params), ctypes.byref(out)))
    return out.value


def xy_group_add(g, params: xy_params, nsweeps: int):
    """Slot id, or None when the request does not fit right now (XY_EBUDGET)."""
    slot = ctypes.c_int32(-1)
    rc = load().xy_group_add(g, ctypes.byref(params), nsweeps, ctypes.byref(slot))
    if rc == XY_EBUDGET:
        return None
    _check(rc)
    return slot.value


def xy_group_round(g, max_sweeps: int) -> int:
    ran = ctypes.c_int64(0)
    _check(load().xy_group_round(g, max_sweeps, ctypes.byref(ran)))
    return ran.value


def xy_group_poll(g, cap: int = 1024):
    out = np.zeros(cap, dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(load().xy_group_poll(g, _ptr(out), cap, ctypes.byref(n)))
    return [int(v) for v in out[:n.value]]


def xy_group_result(g, slot: int):
    """(observables after the latest sweep, beta, mean beta over PCC steps)."""
    last = np.zeros(1, dtype=OBS_DTYPE)
    beta = ctypes.c_double(0.0)
    mean = ctypes.c_double(0.0)
    _check(load().xy_group_result(g, slot, _ptr(last), ctypes.byref(beta), ctypes.byref(mean)))
    return last[0], beta.value, mean.value


def xy_group_get_state(g, slot: int, c: np.ndarray, s: np.ndarray):
    _check(load().xy_group_get_state(g, slot, _ptr(c), _ptr(s)))


def xy_group_release(g, slot: int):
    _check(load().xy_group_release(g, slot))


def xy_group_info(g):
    used = ctypes.c_size_t(0)
    running = ctypes.c_int32(0)
    _check(load().xy_group_info(g, ctypes.byref(used), ctypes.byref(running)))
    return used.value, running.value


def xy_group_free(g):
    _check(load().xy_group_free(g))
