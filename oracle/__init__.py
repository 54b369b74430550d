"""CPU oracle for the Swendsen-Wang / PCC hot path of the 2D classical XY model.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
package never does, and the two share no code.

The arithmetic lives in plain C (``xy_oracle.c``: FP64, breadth-first-search
labelling, its own Philox4x32-10; ``metropolis.c``: an unrelated single-spin
Metropolis chain).  This module compiles them with gcc (``-O2
-ffp-contract=off``, no fast-math) and wraps them with ctypes and numpy.

Every function follows a passage of Komura & Okabe, arXiv:1210.6116:
  * model: Eq. (Hc), periodic L x L square lattice, J = 1;
  * update: the Swendsen-Wang multi-cluster algorithm with Wolff's embedding
    (introduction, the SW / PCC paragraphs);
  * observables: the helicity-modulus definitions of e and s over links in one
    direction, and <m^2>_L = chi / L^2 (equation before Eq. (m2_2r));
  * controller: the generalized PCC rule (compare beta*Upsilon with 0.636508,
    move beta by dbeta), with the window and dbeta of the simulation paragraph.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ("xy_oracle.c", "metropolis.c")
_LIBNAME = "liboracle.so"
_lib = None

OBS_NAMES = ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2")
NOBS = len(OBS_NAMES)
PCC_TARGET = 0.636508  # critical beta*Upsilon with the periodic-boundary winding correction


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into ``oracle/liboracle.so`` with gcc."""
    out = os.path.join(_HERE, _LIBNAME)
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-Wextra", "-o", tmp]
        cmd += [os.path.join(_HERE, s) for s in _SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _stale(path: str) -> bool:
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    return any(os.path.getmtime(os.path.join(_HERE, f)) > t for f in _SOURCES)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # XY_ORACLE_LIB: load another build of these sources (the mutation tests
    # compile deliberately broken copies of the oracle to check that the pins fail)
    path = os.environ.get("XY_ORACLE_LIB") or os.path.join(_HERE, _LIBNAME)
    if not os.environ.get("XY_ORACLE_LIB") and _stale(path):
        build(force=True)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    u32p, u64p, dp, i64p, u8p = (P(ctypes.c_uint32), P(ctypes.c_uint64), P(ctypes.c_double),
                                  P(ctypes.c_int64), P(ctypes.c_uint8))
    i64, u64, u32, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_double
    sig = {
        "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
        "orc_philox4x64_10": (None, [u64p, u64p, u64p]),
        "orc_direction": (None, [u64, u32, u64, dp]),
        "orc_hot_start": (None, [i64, u64, u32, i32, dp, dp]),
        "orc_bonds": (None, [i64, dp, dp, dbl, dp, u64, u32, u64, u8p, u8p, i64p]),
        "orc_label": (i32, [i64, u8p, u8p, i64p]),
        "orc_links": (None, [i64, i64, i64p, u8p, dp, dp, dp, dp, dbl, dp, u64, u32, u64, u8p, i64p]),
        "orc_coin": (i32, [u64, u32, u64, i64]),
        "orc_flip": (None, [i64, i64p, dp, dp, dp, u64, u32, u64, i32]),
        "orc_renorm": (None, [i64, dp, dp, i32]),
        "orc_measure": (None, [i64, dp, dp, dbl, dp]),
        "orc_sweep": (i32, [i64, dp, dp, dbl, u64, u32, u64, i32, dp, i64p, u8p, u8p, i64p]),
        "orc_run": (i32, [i64, dp, dp, dbl, u64, u32, u64, i64, i32, dp, i64p]),
        "orc_pcc_run": (i32, [i64, dp, dp, dp, u64, u32, u64, i64, i64, dbl, dbl, i64, dbl, i64,
                              i32, dp, dp]),
        "orc_wrap": (i32, [i64, u8p, u8p, P(ctypes.c_int)]),
        "orc_pcc_perc_run": (i32, [i64, dp, dp, dp, u64, u32, u64, i64, i64, dbl, dbl, i64, dbl, i64,
                                   i32, dp, dp, P(ctypes.c_int32)]),
        "metro_run": (dbl, [i64, dbl, dbl, u64, i64, i64, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ----------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                              _ptr(out, ctypes.c_uint32))
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    """Philox4x64-10 block: counter (4 x u64), key (2 x u64) -> 4 x u64."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(_ptr(c, ctypes.c_uint64), _ptr(k, ctypes.c_uint64),
                              _ptr(out, ctypes.c_uint64))
    return out


def direction(seed: int, rep: int, t: int) -> np.ndarray:
    """Mirror direction r (unit 2-vector, FP64) of sweep t."""
    r = np.zeros(2)
    _load().orc_direction(seed, rep, t, _ptr(r, ctypes.c_double))
    return r


def coin(seed: int, rep: int, t: int, root: int) -> int:
    """Flip coin (0 or 1) of the cluster with canonical root `root` in sweep t."""
    return int(_load().orc_coin(seed, rep, t, root))


# ------------------------------------------------------------------------ stages
def hot_start(L: int, seed: int, rep: int = 0, storage32: bool = True):
    """Uniform-angle start: returns (cos, sin) FP64 arrays of N = L*L values."""
    N = L * L
    c = np.zeros(N)
    s = np.zeros(N)
    _load().orc_hot_start(L, seed, rep, int(storage32), _ptr(c, ctypes.c_double),
                          _ptr(s, ctypes.c_double))
    return c, s


def bonds(L, c, s, beta, r, seed, rep, t):
    """Active x- and y-links (uint8 per site) and the near-tie count."""
    N = L * L
    c = np.ascontiguousarray(c, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    bx = np.zeros(N, dtype=np.uint8)
    by = np.zeros(N, dtype=np.uint8)
    ties = ctypes.c_int64(0)
    _load().orc_bonds(L, _ptr(c, ctypes.c_double), _ptr(s, ctypes.c_double), beta,
                      _ptr(r, ctypes.c_double), seed, rep, t, _ptr(bx, ctypes.c_uint8),
                      _ptr(by, ctypes.c_uint8), ctypes.byref(ties))
    return bx, by, int(ties.value)


def links(L, site, dirs, ci, si, cj, sj, beta, r, seed, rep, t):
    """Decisions (uint8) of the links site[k] -> right (dirs[k] = 0) or down
    (dirs[k] = 1), from the given end spins; and the near-tie count."""
    site = np.ascontiguousarray(site, dtype=np.int64)
    n = site.size
    dirs = np.ascontiguousarray(dirs, dtype=np.uint8)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (ci, si, cj, sj)]
    assert dirs.size == n and all(a.size == n for a in arrs)
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(n, dtype=np.uint8)
    ties = ctypes.c_int64(0)
    _load().orc_links(L, n, _ptr(site, ctypes.c_int64), _ptr(dirs, ctypes.c_uint8),
                      *[_ptr(a, ctypes.c_double) for a in arrs], beta, _ptr(r, ctypes.c_double),
                      seed, rep, t, _ptr(out, ctypes.c_uint8), ctypes.byref(ties))
    return out, int(ties.value)


def label(L, bx, by) -> np.ndarray:
    """Canonical (minimum-site) cluster label of every site, by BFS."""
    N = L * L
    bx = np.ascontiguousarray(bx, dtype=np.uint8)
    by = np.ascontiguousarray(by, dtype=np.uint8)
    out = np.zeros(N, dtype=np.int64)
    if _load().orc_label(L, _ptr(bx, ctypes.c_uint8), _ptr(by, ctypes.c_uint8),
                         _ptr(out, ctypes.c_int64)) != 0:
        raise MemoryError("oracle labelling ran out of memory")
    return out


def wrap(L, bx, by) -> int:
    """Wrapping of the clusters of a link set: bit 0 if some cluster winds
    around the periodic lattice along x, bit 1 along y."""
    bx = np.ascontiguousarray(bx, dtype=np.uint8)
    by = np.ascontiguousarray(by, dtype=np.uint8)
    w = ctypes.c_int(0)
    if _load().orc_wrap(L, _ptr(bx, ctypes.c_uint8), _ptr(by, ctypes.c_uint8), ctypes.byref(w)) != 0:
        raise MemoryError("oracle wrapping check ran out of memory")
    return int(w.value)


def flip(L, lab, c, s, r, seed, rep, t, storage32=True):
    """Reflect every cluster whose coin is set; returns new (cos, sin)."""
    c = np.array(c, dtype=np.float64)
    s = np.array(s, dtype=np.float64)
    lab = np.ascontiguousarray(lab, dtype=np.int64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    _load().orc_flip(L, _ptr(lab, ctypes.c_int64), _ptr(c, ctypes.c_double),
                     _ptr(s, ctypes.c_double), _ptr(r, ctypes.c_double), seed, rep, t,
                     int(storage32))
    return c, s


def measure(L, c, s, beta) -> np.ndarray:
    """Observables (E, m2, ex, sx, ey, sy, ups_x, mk2) of one configuration."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    obs = np.zeros(NOBS)
    _load().orc_measure(L, _ptr(c, ctypes.c_double), _ptr(s, ctypes.c_double), beta,
                        _ptr(obs, ctypes.c_double))
    return obs


# ------------------------------------------------------------------------ chains
@dataclass
class Lattice:
    """One L x L lattice driven by the oracle (state, beta, seed, replica, sweep)."""

    L: int
    beta: float
    seed: int
    rep: int = 0
    storage32: bool = True
    t: int = 0
    c: np.ndarray = field(default=None, repr=False)
    s: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        if self.c is None:
            self.c, self.s = hot_start(self.L, self.seed, self.rep, self.storage32)
        else:
            self.c = np.array(self.c, dtype=np.float64)
            self.s = np.array(self.s, dtype=np.float64)

    def sweep_detail(self):
        """One sweep, returning (obs, ties, bx, by, labels) of that sweep."""
        N = self.L * self.L
        bx = np.zeros(N, dtype=np.uint8)
        by = np.zeros(N, dtype=np.uint8)
        lab = np.zeros(N, dtype=np.int64)
        obs = np.zeros(NOBS)
        ties = ctypes.c_int64(0)
        rc = _load().orc_sweep(self.L, _ptr(self.c, ctypes.c_double), _ptr(self.s, ctypes.c_double),
                               self.beta, self.seed, self.rep, self.t, int(self.storage32),
                               _ptr(obs, ctypes.c_double), ctypes.byref(ties),
                               _ptr(bx, ctypes.c_uint8), _ptr(by, ctypes.c_uint8),
                               _ptr(lab, ctypes.c_int64))
        if rc != 0:
            raise MemoryError("oracle sweep ran out of memory")
        self.t += 1
        return obs, int(ties.value), bx, by, lab

    def run(self, n: int):
        """n sweeps; returns (trace[n, NOBS], ties[n])."""
        trace = np.zeros((n, NOBS))
        ties = np.zeros(n, dtype=np.int64)
        rc = _load().orc_run(self.L, _ptr(self.c, ctypes.c_double), _ptr(self.s, ctypes.c_double),
                             self.beta, self.seed, self.rep, self.t, n, int(self.storage32),
                             _ptr(trace, ctypes.c_double), _ptr(ties, ctypes.c_int64))
        if rc != 0:
            raise MemoryError("oracle run ran out of memory")
        self.t += n
        return trace, ties

    def pcc(self, nsteps: int, window: int, dbeta0: float, dbeta_min: float = 0.0,
            halve_every: int = 0, target: float = PCC_TARGET, k0: int = 0):
        """nsteps PCC steps; returns (beta after each step, beta*Upsilon of each window)."""
        beta = ctypes.c_double(self.beta)
        btr = np.zeros(nsteps)
        butr = np.zeros(nsteps)
        rc = _load().orc_pcc_run(self.L, _ptr(self.c, ctypes.c_double), _ptr(self.s, ctypes.c_double),
                                 ctypes.byref(beta), self.seed, self.rep, self.t, nsteps, window,
                                 dbeta0, dbeta_min, halve_every, target, k0, int(self.storage32),
                                 _ptr(btr, ctypes.c_double), _ptr(butr, ctypes.c_double))
        if rc != 0:
            raise MemoryError("oracle PCC run ran out of memory")
        self.beta = beta.value
        self.t += nsteps * window
        return btr, butr

    def pcc_perc(self, nsteps: int, window: int, dbeta0: float, dbeta_min: float = 0.0,
                 halve_every: int = 0, target: float = 0.5, k0: int = 0):
        """nsteps steps of the percolation PCC rule; returns (beta after each
        step, wrapping fraction of each window, wrap bits of every sweep)."""
        beta = ctypes.c_double(self.beta)
        btr = np.zeros(nsteps)
        ptr_ = np.zeros(nsteps)
        wtr = np.zeros(nsteps * window, dtype=np.int32)
        rc = _load().orc_pcc_perc_run(self.L, _ptr(self.c, ctypes.c_double), _ptr(self.s, ctypes.c_double),
                                      ctypes.byref(beta), self.seed, self.rep, self.t, nsteps, window,
                                      dbeta0, dbeta_min, halve_every, target, k0, int(self.storage32),
                                      _ptr(btr, ctypes.c_double), _ptr(ptr_, ctypes.c_double),
                                      _ptr(wtr, ctypes.c_int32))
        if rc != 0:
            raise MemoryError("oracle PCC run ran out of memory")
        self.beta = beta.value
        self.t += nsteps * window
        return btr, ptr_, wtr


def metropolis(L: int, beta: float, nsweeps: int, ntherm: int = 1000, seed: int = 1,
               delta: float = 2.0, theta0=None):
    """Independent Metropolis chain; returns (trace[nsweeps, 5], acceptance, theta).

    Columns of trace: E, m2, ex, sx, ups_x (same definitions as the SW oracle).
    """
    th = np.zeros(L * L) if theta0 is None else np.array(theta0, dtype=np.float64)
    trace = np.zeros((nsweeps, 5))
    acc = _load().metro_run(L, beta, delta, seed, ntherm, nsweeps, _ptr(th, ctypes.c_double),
                            _ptr(trace, ctypes.c_double))
    return trace, acc, th
