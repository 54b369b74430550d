"""Seeded synthetic inputs for the 2D XY Swendsen-Wang / PCC workloads.

This module is the only code that both the CPU oracle's tests and the HIP path's
tests use.  It holds none of the method's arithmetic: it only draws seeded
numbers with numpy and shapes them into arrays and tables (random FP32 spin
states, bond patterns for the labelling step, replica tables for batched runs,
request traces for the serving loop).  Random numbers the method itself draws
(directions, bond uniforms, coins, the hot start) are not made here; each side
computes them from its own Philox4x32-10.
"""
from __future__ import annotations

import numpy as np

# Seeds and shapes of the standard workloads.
SEED_L64 = 0x12106116       # L = 64, beta = 1.12, 1000 sweeps
SEED_L4096 = 0x12106117     # L = 4096, beta = 1.12, 200 + 1000 sweeps
SEED_BATCH = 0x12106118     # 512 replicas, L log-uniform over 64..2048
SEED_L65536 = 0x12106119    # L = 65536 PCC run
SEED_SERVE = 0x1211         # serving trace
BETA_FIXED = 1.12


def random_spins(L: int, seed: int):
    """Independent uniform angles, returned as FP32 (cos, sin) planes of N = L*L."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, 2.0 * np.pi, size=L * L)
    return np.cos(th).astype(np.float32), np.sin(th).astype(np.float32)


def aligned_spins(L: int, angle: float = 0.0):
    """Every spin at the same angle (cold start), FP32 (cos, sin)."""
    N = L * L
    return (np.full(N, np.cos(angle), dtype=np.float32), np.full(N, np.sin(angle), dtype=np.float32))


def random_bonds(L: int, p: float, seed: int):
    """Bernoulli(p) x- and y-links, uint8 per site."""
    rng = np.random.default_rng(seed)
    N = L * L
    return ((rng.random(N) < p).astype(np.uint8), (rng.random(N) < p).astype(np.uint8))


def pattern_bonds(L: int, kind: str):
    """Adversarial link patterns for the labelling step (uint8 bx, by per site).

    kinds: 'none', 'all', 'comb' (full rows joined by one column), 'spiral' (a
    single path winding inwards), 'checker' (isolated pairs on a checkerboard),
    'wrap' (a strip that only closes through the periodic x boundary),
    'snake' (boustrophedon path through every site), 'vbars' (vertical bars).
    """
    N = L * L
    bx = np.zeros((L, L), dtype=np.uint8)
    by = np.zeros((L, L), dtype=np.uint8)
    if kind == "none":
        pass
    elif kind == "all":
        bx[:] = 1
        by[:] = 1
    elif kind == "comb":
        bx[:, : L - 1] = 1
        by[:, 0] = 1
        by[L - 1, 0] = 0
    elif kind == "checker":
        yy, xx = np.mgrid[0:L, 0:L]
        bx[((xx + yy) % 2 == 0) & (xx < L - 1)] = 1
    elif kind == "wrap":
        bx[L // 2, :] = 1
        bx[L // 2, L // 2 - 1] = 0
    elif kind == "snake":
        for y in range(L):
            bx[y, : L - 1] = 1
            if y < L - 1:
                by[y, L - 1 if y % 2 == 0 else 0] = 1
    elif kind == "vbars":
        by[: L - 1, ::2] = 1
    elif kind == "spiral":
        grid = np.zeros((L, L), dtype=bool)
        x = y = 0
        dx, dy = 1, 0
        lo_x, hi_x, lo_y, hi_y = 0, L - 1, 0, L - 1
        grid[0, 0] = True
        while True:
            nx, ny = x + dx, y + dy
            if not (lo_x <= nx <= hi_x and lo_y <= ny <= hi_y) or grid[ny, nx]:
                # turn clockwise, tightening the ring every other turn
                if (dx, dy) == (1, 0):
                    dx, dy = 0, 1
                    lo_y += 1
                elif (dx, dy) == (0, 1):
                    dx, dy = -1, 0
                    hi_x -= 1
                elif (dx, dy) == (-1, 0):
                    dx, dy = 0, -1
                    hi_y -= 1
                else:
                    dx, dy = 1, 0
                    lo_x += 1
                nx, ny = x + dx, y + dy
                if not (lo_x <= nx <= hi_x and lo_y <= ny <= hi_y) or grid[ny, nx]:
                    break
            if dx == 1:
                bx[y, x] = 1
            elif dx == -1:
                bx[ny, nx] = 1
            elif dy == 1:
                by[y, x] = 1
            else:
                by[ny, nx] = 1
            x, y = nx, ny
            grid[y, x] = True
    else:
        raise ValueError("unknown pattern %r" % kind)
    return bx.reshape(N), by.reshape(N)


PATTERNS = ("none", "all", "comb", "checker", "wrap", "snake", "vbars", "spiral")


def batched_replicas(n: int = 512, seed: int = SEED_BATCH, jmax: int = 5, lmin_log2: int = 6,
                     beta_lo: float = 1.0, beta_hi: float = 1.2):
    """Replica table of the batched workload.

    L_k = 2^(lmin_log2 + j_k) with j_k uniform on {0..jmax} (log-uniform sizes),
    beta_k uniform on [beta_lo, beta_hi]; every replica shares the Philox key
    `seed` and uses its index k as its stream id.  Returns a list of dicts.
    """
    rng = np.random.default_rng(seed)
    j = rng.integers(0, jmax + 1, size=n)
    betas = rng.uniform(beta_lo, beta_hi, size=n)
    return [dict(L=int(2 ** (lmin_log2 + int(j[k]))), beta=float(betas[k]), seed=int(seed), rep=k)
            for k in range(n)]


def serving_trace(n_requests: int = 200, rate: float = 20.0, seed: int = SEED_SERVE,
                  lmin_log2: int = 8, jmax: int = 5, sweeps_lo: int = 1000, sweeps_hi: int = 10000):
    """Poisson request trace of the serving workload.

    Arrival gaps ~ Exp(rate); L = 2^(lmin_log2 + j), j uniform on {0..jmax};
    sweeps uniform on {sweeps_lo..sweeps_hi}; a 64-bit Philox key per request.
    Returns a list of dicts with keys arrival (s), L, sweeps, seed, beta0.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    j = rng.integers(0, jmax + 1, size=n_requests)
    sweeps = rng.integers(sweeps_lo, sweeps_hi + 1, size=n_requests)
    seeds = rng.integers(0, 2 ** 63 - 1, size=n_requests, dtype=np.int64)
    return [dict(arrival=float(arrivals[k]), L=int(2 ** (lmin_log2 + int(j[k]))),
                 sweeps=int(sweeps[k]), seed=int(seeds[k]), beta0=1.0) for k in range(n_requests)]
