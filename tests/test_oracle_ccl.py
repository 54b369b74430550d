"""Pins of the oracle's connected-component labelling (BFS, canonical min-site labels).

Checked against brute force on every link subset of the L = 2 lattice and against
an unrelated union-find written here, on random and adversarial link sets.
"""
import itertools

import numpy as np
import pytest

import oracle
import xyworkloads as wl


def _neighbours(L):
    N = L * L
    idx = np.arange(N)
    x, y = idx % L, idx // L
    return y * L + (x + 1) % L, ((y + 1) % L) * L + x


def _closure_labels(L, bx, by):
    """Components by transitive closure of the adjacency matrix (tiny L only)."""
    N = L * L
    right, down = _neighbours(L)
    A = np.eye(N, dtype=bool)
    for i in range(N):
        if bx[i]:
            A[i, right[i]] = A[right[i], i] = True
        if by[i]:
            A[i, down[i]] = A[down[i], i] = True
    for k in range(N):  # Warshall
        A = A | (A[:, k:k + 1] & A[k:k + 1, :])
    return np.array([int(np.flatnonzero(A[i])[0]) for i in range(N)])


def _unionfind_labels(L, bx, by):
    N = L * L
    right, down = _neighbours(L)
    parent = list(range(N))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i in range(N):
        for on, j in ((bx[i], right[i]), (by[i], down[i])):
            if on:
                a, b = find(i), find(int(j))
                if a != b:
                    parent[max(a, b)] = min(a, b)
    roots = np.array([find(i) for i in range(N)])
    # canonical label = minimum site of the component
    mins = {}
    for i, r in enumerate(roots):
        mins.setdefault(int(r), i)
    return np.array([mins[int(r)] for r in roots])


def test_l2_every_link_subset():
    L = 2
    for bits in itertools.product((0, 1), repeat=8):
        bx = np.array(bits[:4], dtype=np.uint8)
        by = np.array(bits[4:], dtype=np.uint8)
        assert np.array_equal(oracle.label(L, bx, by), _closure_labels(L, bx, by)), bits


@pytest.mark.parametrize("L", [4, 8, 16, 64])
@pytest.mark.parametrize("p", [0.0, 0.3, 0.5, 0.7, 1.0])
def test_random_links_vs_union_find(L, p):
    bx, by = wl.random_bonds(L, p, seed=1000 + L + int(p * 100))
    lab = oracle.label(L, bx, by)
    assert np.array_equal(lab, _unionfind_labels(L, bx, by))
    if L <= 8:
        assert np.array_equal(lab, _closure_labels(L, bx, by))


@pytest.mark.parametrize("L", [2, 4, 8, 32])
@pytest.mark.parametrize("kind", wl.PATTERNS)
def test_adversarial_patterns(L, kind):
    bx, by = wl.pattern_bonds(L, kind)
    lab = oracle.label(L, bx, by)
    assert np.array_equal(lab, _unionfind_labels(L, bx, by))
    # canonical: every label is the smallest site carrying it, and labels <= index
    assert np.all(lab <= np.arange(L * L))
    assert np.all(lab[lab] == lab)
