"""The host cluster search used by the full-size over-merge check, pinned on the
CPU against the oracle's labelling of whole lattices (random links near the
bond-percolation threshold, so that clusters of every size occur, and link
patterns that close only through the periodic boundary)."""
import numpy as np
import torch

import oracle
import xyworkloads as wl
from clusters import host_cluster


def _words(b: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.packbits(b, bitorder="little").view("<u4").astype(np.uint32).view(np.int32))


def test_host_cluster_matches_oracle_labels():
    L = 512
    bx, by = wl.random_bonds(L, 0.45, 2024)
    lab = oracle.label(L, bx, by)
    sizes = np.bincount(lab, minlength=L * L)
    wbx, wby = _words(bx), _words(by)
    rng = np.random.default_rng(7)
    decided = 0
    for site in rng.integers(0, L * L, 60):
        m = host_cluster(wbx, wby, L, int(site), radii=(32, 64, 128))
        if m is None:
            continue
        decided += 1
        assert m.size == sizes[lab[site]]
        assert int(m.min()) == lab[site]
        assert np.all(lab[m] == lab[site])
    assert decided >= 40


def test_host_cluster_across_the_periodic_boundary():
    L = 256
    bx = np.zeros((L, L), np.uint8)
    by = np.zeros((L, L), np.uint8)
    bx[5, L - 3:] = 1          # (5, L-3) .. (5, L-1) -> (5, 0), then on to (5, 2)
    bx[5, :2] = 1
    by[L - 1, 7] = 1           # (L-1, 7) -> (0, 7)
    by[0, 7] = 1               # (0, 7) -> (1, 7)
    bx, by = bx.ravel(), by.ravel()
    lab = oracle.label(L, bx, by)
    for site, expect in ((5 * L + 1, 6), (0 * L + 7, 3)):
        m = host_cluster(_words(bx), _words(by), L, site, radii=(32,))
        assert m is not None and m.size == expect
        assert np.all(lab[m] == lab[site]) and int(m.min()) == lab[site]
