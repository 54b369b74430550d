"""Pins of the oracle's wrapping check (the observation of the original,
percolation-driven PCC rule: do the clusters percolate?).

On the periodic lattice a cluster percolates along x when it holds a closed
path of active links whose winding number along x is not zero.  The oracle
finds this with unwrapped coordinates in a breadth-first search.  Pinned here
by
  * hand-built link sets at L = 4 and 8 whose windings are known by
    construction (lines, closed staircases, rings, a comb that touches every
    column without winding, a path one link short of closing);
  * an unrelated characterisation, counted with a library graph routine: lift
    the link set to the k-fold cover of the torus along x (a kL x L torus,
    k a prime above L).  A cluster whose closed paths have x-windings with
    greatest common divisor g lifts to gcd(g, k) clusters; g <= L < k, so the
    lift of every cluster is k separate copies exactly when no cluster winds
    along x.  Checked on every link subset of L = 2 and on random link sets at
    L = 3, 4, 8 and 16 around the density where wrapping sets in;
  * symmetries: translating the link set keeps the bits, transposing the
    lattice swaps them.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle

WX, WY = 1, 2


def _empty(L):
    return np.zeros(L * L, np.uint8), np.zeros(L * L, np.uint8)


def _site(L, x, y):
    return (y % L) * L + (x % L)


def _path(L, steps, x0=0, y0=0):
    """Link planes of a walk from (x0, y0) along steps in 'RLDU' (right, left, down, up)."""
    bx, by = _empty(L)
    x, y = x0, y0
    for s in steps:
        if s == "R":
            bx[_site(L, x, y)] = 1
            x += 1
        elif s == "L":
            x -= 1
            bx[_site(L, x, y)] = 1
        elif s == "D":
            by[_site(L, x, y)] = 1
            y += 1
        elif s == "U":
            y -= 1
            by[_site(L, x, y)] = 1
    return bx, by


HAND = [
    # (name, L, builder, expected bits)
    ("nothing", 4, lambda L: _empty(L), 0),
    ("row_closed", 4, lambda L: _path(L, "RRRR", 0, 1), WX),
    ("row_one_short", 8, lambda L: _path(L, "R" * 7, 0, 3), 0),
    ("column_closed", 8, lambda L: _path(L, "D" * 8, 5, 0), WY),
    ("staircase_1_1", 4, lambda L: _path(L, "RD" * 4), WX | WY),
    ("staircase_open", 8, lambda L: _path(L, "RRRRD" * 4, 0, 0), 0),
    ("staircase_2_1_closed", 4, lambda L: _path(L, "RRD" * 4, 0, 0), WX | WY),
    ("diagonal_plus_row", 4, lambda L: _path(L, "RD" * 4 + "RRRR", 0, 0), WX | WY),
    ("ring_around_plaquettes", 8, lambda L: _path(L, "RRRDDDLLLUUU", 2, 2), 0),
    ("comb_every_column", 8, lambda L: _path(L, "RDRURDRURDRURD", 0, 0), 0),
    ("snake_every_row", 8, lambda L: _path(L, "DRDLDRDLDRDLD", 3, 0), 0),
    ("back_and_forth", 4, lambda L: _path(L, "RRRLLL", 0, 0), 0),
    ("two_rows_one_closed", 8, lambda L: _merge(_path(L, "R" * 8, 0, 2), _path(L, "R" * 6, 0, 6)), WX),
    ("cross_of_lines", 8, lambda L: _merge(_path(L, "R" * 8, 0, 4), _path(L, "D" * 8, 4, 0)), WX | WY),
]


def _merge(a, b):
    return np.maximum(a[0], b[0]), np.maximum(a[1], b[1])


def test_hand_built_sets():
    for name, L, build, want in HAND:
        bx, by = build(L)
        assert oracle.wrap(L, bx, by) == want, name


def test_closed_2_1_staircase_winds_both_ways():
    bx, by = _path(4, "RRD" * 2, 0, 0)
    # 'RRD' x 2 ends at (4, 2) = (0, 2): not closed in y yet -> no winding
    assert oracle.wrap(4, bx, by) == 0
    bx, by = _path(4, "RRD" * 4, 0, 0)
    # (8, 4): closed, windings (2, 1)
    assert oracle.wrap(4, bx, by) == WX | WY


def _components_of_lift(L, bx, by, k, along):
    """Connected components of the link set lifted to the k-fold cover of the
    torus along x (a kL x L torus) or along y (L x kL)."""
    W, H = (k * L, L) if along == "x" else (L, k * L)
    rows, cols = [], []
    for c in range(k):
        for y in range(L):
            for x in range(L):
                i = y * L + x
                X, Y = (c * L + x, y) if along == "x" else (x, c * L + y)
                a = Y * W + X
                if bx[i]:
                    rows.append(a)
                    cols.append(Y * W + (X + 1) % W)
                if by[i]:
                    rows.append(a)
                    cols.append(((Y + 1) % H) * W + X)
    n = W * H
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    return connected_components(g, directed=False)[0]


def _components(L, bx, by):
    return _components_of_lift(L, bx, by, 1, "x")


def _next_prime(n):
    p = n + 1
    while any(p % d == 0 for d in range(2, int(p ** 0.5) + 1)):
        p += 1
    return p


def _by_cover(L, bx, by):
    k = _next_prime(L)
    base = _components(L, bx, by)
    bits = 0
    if _components_of_lift(L, bx, by, k, "x") < k * base:
        bits |= WX
    if _components_of_lift(L, bx, by, k, "y") < k * base:
        bits |= WY
    return bits


def test_l2_every_link_subset_against_the_cover():
    L = 2
    for mask in range(256):
        bits = [(mask >> j) & 1 for j in range(8)]
        bx = np.array(bits[:4], np.uint8)
        by = np.array(bits[4:], np.uint8)
        assert oracle.wrap(L, bx, by) == _by_cover(L, bx, by), mask


@pytest.mark.parametrize("L,n", [(3, 300), (4, 300), (8, 150), (16, 40)])
def test_random_sets_against_the_cover(L, n):
    rng = np.random.default_rng(1000 + L)
    seen = set()
    for trial in range(n):
        p = rng.uniform(0.3, 0.75)
        bx = (rng.random(L * L) < p).astype(np.uint8)
        by = (rng.random(L * L) < p).astype(np.uint8)
        got = oracle.wrap(L, bx, by)
        assert got == _by_cover(L, bx, by), (L, trial)
        seen.add(got)
    assert seen == {0, WX, WY, WX | WY}, seen  # every outcome occurs


def test_symmetries():
    rng = np.random.default_rng(7)
    L = 8
    for _ in range(50):
        bx = (rng.random(L * L) < 0.5).astype(np.uint8)
        by = (rng.random(L * L) < 0.5).astype(np.uint8)
        w = oracle.wrap(L, bx, by)
        sx, sy = rng.integers(0, L, 2)
        tx = np.roll(bx.reshape(L, L), (sy, sx), axis=(0, 1)).ravel()
        ty = np.roll(by.reshape(L, L), (sy, sx), axis=(0, 1)).ravel()
        assert oracle.wrap(L, tx, ty) == w
        # transpose: x-links become y-links
        assert oracle.wrap(L, by.reshape(L, L).T.ravel().copy(), bx.reshape(L, L).T.ravel().copy()) == \
            ((w & WX) << 1) | ((w & WY) >> 1)


def test_percolation_pcc_direction_of_steps():
    """beta = 0: no links, nothing wraps, beta must rise every step; very large
    beta: the clusters span the lattice, beta must fall."""
    lat = oracle.Lattice(L=8, beta=0.0, seed=11)
    betas, p, w = lat.pcc_perc(5, 4, 0.01, target=0.5)
    assert np.all(p == 0.0) and np.all(w == 0)
    assert np.allclose(betas, 0.01 * np.arange(1, 6))
    lat = oracle.Lattice(L=8, beta=5.0, seed=12)
    lat.run(20)
    betas, p, w = lat.pcc_perc(5, 4, 0.01, target=0.5)
    assert np.all(p >= 0.5)
    assert np.allclose(betas, 5.0 - 0.01 * np.arange(1, 6))


def test_percolation_pcc_fixed_point():
    """The percolation rule settles where the wrapping probability is the
    target: started far away on either side, a W = 20 run at L = 8 ends at the
    same beta*, and fixed-beta runs just below / above beta* wrap less / more
    often than half of the time."""
    ends = []
    for beta0, seed in ((0.4, 21), (1.6, 22)):
        lat = oracle.Lattice(L=8, beta=beta0, seed=seed)
        betas, p, w = lat.pcc_perc(150, 20, 0.02, dbeta_min=0.0025, halve_every=30, target=0.5)
        ends.append(betas[-40:].mean())
    assert abs(ends[0] - ends[1]) < 0.05, ends
    bstar = 0.5 * (ends[0] + ends[1])

    def wrap_rate(beta, seed):
        lat = oracle.Lattice(L=8, beta=beta, seed=seed)
        lat.run(50)
        _, p, _ = lat.pcc_perc(1, 3000, 0.0, target=0.5)  # dbeta 0: a fixed-beta run that records wrapping
        return p[0]

    assert wrap_rate(bstar - 0.15, 31) < 0.5 < wrap_rate(bstar + 0.15, 32)
