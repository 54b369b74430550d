"""Host breadth-first search of one cluster of a periodic L x L lattice from its
link bit planes, read through windows around a site (for lattices too large to
copy to the host whole).  Independent of the labelling kernels and of the
oracle's labelling: a library BFS over the window's link graph."""
import numpy as np
import torch
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import breadth_first_order


def window_bits(words: torch.Tensor, L: int, y0: int, xs: int, R: int) -> np.ndarray:
    """Bits of the 2R x 2R window with rows y0 - R .. y0 + R - 1 and columns
    xs .. xs + 2R - 1 (periodic) of a plane of little-endian 32-bit words (bit
    i of word i // 32 belongs to site i = y L + x); xs and R multiples of 32."""
    W = L // 32
    rows = torch.arange(y0 - R, y0 + R, device=words.device) % L
    cols = torch.arange(xs // 32, xs // 32 + 2 * R // 32, device=words.device) % W
    w = words.view(L, W).index_select(0, rows).index_select(1, cols).cpu().numpy()
    bits = np.unpackbits(np.ascontiguousarray(w).view("<u4").view(np.uint8), axis=1, bitorder="little")
    return bits.reshape(2 * R, 2 * R)


def host_cluster(bx: torch.Tensor, by: torch.Tensor, L: int, site: int, radii=(128, 512, 2048)):
    """Global site indices of the cluster of `site` (x-link plane bx: site i to
    its right neighbour, y-link plane by: to the one below), found by BFS over
    the active links inside windows of growing radius around the site; None if
    the cluster reaches the edge of the largest window (or the window would
    wrap around the lattice)."""
    y, x = divmod(site, L)
    for R in radii:
        if 2 * R > L:
            break
        xs = (x - R) // 32 * 32  # first window column: a word boundary at or left of x - R
        wx = window_bits(bx, L, y, xs, R)
        wy = window_bits(by, L, y, xs, R)
        n = 2 * R
        idx = np.arange(n * n).reshape(n, n)
        a_x = idx[:, :-1][wx[:, :-1] == 1]  # (r, c) -> (r, c + 1) inside the window
        a_y = idx[:-1, :][wy[:-1, :] == 1]  # (r, c) -> (r + 1, c)
        a = np.concatenate([a_x, a_y])
        b = np.concatenate([a_x + 1, a_y + n])
        g = coo_matrix((np.ones(a.size, dtype=np.int8), (a, b)), shape=(n * n, n * n)).tocsr()
        order = breadth_first_order(g, R * n + (x - xs), directed=False, return_predecessors=False)
        r, c = np.divmod(order, n)
        if r.min() == 0 or c.min() == 0 or r.max() == n - 1 or c.max() == n - 1:
            continue  # on the window's edge: the cluster may continue outside
        return ((y - R + r) % L).astype(np.int64) * L + (xs + c) % L
    return None
