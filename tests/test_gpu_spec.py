"""Sweeps that end a PCC window: the flip activates the next sweep's links for
both betas the PCC step may choose (TILE_SPEC), and the next sweep labels the
links of the chosen beta (TILE_PLSEL) instead of activating them again.

Bar: links, labels, spins and beta bit-exact with the oracle's PCC chain, near
ties equal, observables 1e-10 per site; and identical bit for bit to the same
steps taken one call at a time (each call ends with a plain flip, so the next
activates its links from the spins).  Cases: window 1 (every sweep moves
beta) and windows of several sweeps, the halving schedule, tile heights 16 /
32 / 64, lattices narrower than a tile, 64-bit site indices, and a batch
whose replicas sit at different points of their windows."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NAMES = ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2")


def _xy():
    import paper_1210_6116_amd as xy
    return xy


@pytest.mark.parametrize("L,rows,window", [(8, 0, 1), (32, 16, 1), (64, 32, 1), (128, 64, 2), (256, 16, 3),
                                           (256, 32, 1)])
def test_pcc_chain_against_oracle(L, rows, window):
    xy = _xy()
    seed, beta0, nsteps = 0x5BEC + L, 1.0, 24
    print("spec PCC L=%d rows=%d window=%d" % (L, rows, window), flush=True)
    lat = xy.Lattices(dict(L=L, beta=beta0, seed=seed, tile_rows=rows))
    m = lat.pcc(nsteps, window, 0.02, dbeta_min=0.004, halve_every=6, means=True)
    orc = oracle.Lattice(L=L, beta=beta0, seed=seed, storage32=True)
    b_o, bu_o = orc.pcc(nsteps, window, 0.02, dbeta_min=0.004, halve_every=6)
    assert np.array_equal(m["beta"][:, 0], b_o)
    c, s = lat.get_state()
    assert np.array_equal(c.astype(np.float64), orc.c) and np.array_equal(s.astype(np.float64), orc.s)
    # one more sweep on both sides at the final beta: links and labels
    lat.sweep(1)
    orc.beta = float(b_o[-1])
    obs, ties, bx, by, lab = orc.sweep_detail()
    gx, gy = lat.bonds()
    assert np.array_equal(gx, bx) and np.array_equal(gy, by)
    assert np.array_equal(lat.labels(), lab)
    lat.close()


def test_one_call_equals_step_by_step():
    """The window-1 chain in one call (flips with both candidates' links) and
    step by step (a plain flip at the end of every call): every per-step
    window mean, near-tie count and the final state bit-identical."""
    xy = _xy()
    spec = dict(L=512, beta=1.05, seed=0xACE, tile_rows=32)
    a = xy.Lattices(spec)
    b = xy.Lattices(spec)
    ma = a.pcc(30, 1, 0.01, dbeta_min=0.002, halve_every=5, means=True)
    mb = np.concatenate([b.pcc(1, 1, 0.01, dbeta_min=0.002, halve_every=5, means=True) for _ in range(30)])
    # the halving schedule counts steps on the device, so both runs agree on it
    for name in NAMES + ("beta",):
        assert np.array_equal(ma[name], mb[name]), name
    ca, sa = a.get_state()
    cb, sb = b.get_state()
    assert np.array_equal(ca, cb) and np.array_equal(sa, sb)
    assert np.array_equal(a.labels(), b.labels())
    ta = a.sweep(1, trace=True)
    tb = b.sweep(1, trace=True)
    assert int(ta[0, 0]["near_ties"]) == int(tb[0, 0]["near_ties"])
    a.close()
    b.close()


def test_wide_index_chain(monkeypatch):
    """The 64-bit site-index kernels (those of the 2^32-site lattice) on a small
    lattice, window 1: beta trace and state bit-exact with the oracle."""
    monkeypatch.setenv("XY_WIDE_INDEX", "1")
    xy = _xy()
    L, seed = 128, 0x77
    lat = xy.Lattices(dict(L=L, beta=1.0, seed=seed, label_bits=64))
    m = lat.pcc(16, 1, 0.01, dbeta_min=0.002, halve_every=4, means=True)
    orc = oracle.Lattice(L=L, beta=1.0, seed=seed, storage32=True)
    b_o, _ = orc.pcc(16, 1, 0.01, dbeta_min=0.002, halve_every=4)
    assert np.array_equal(m["beta"][:, 0], b_o)
    c, s = lat.get_state()
    assert np.array_equal(c.astype(np.float64), orc.c) and np.array_equal(s.astype(np.float64), orc.s)
    lat.close()


def test_group_mixed_windows_against_oracle():
    """A serving group with window 3 and rounds of 4 sweeps whose requests start
    at different rounds (4 sweeps apart: their windows end at different
    sweeps), so that at most sweeps only some replicas end a window (the others
    keep beta and take the first candidate).  Each request's final beta and
    state equal the oracle's chain."""
    xy = _xy()
    from paper_1210_6116_amd.serve import Group
    pcc = xy.xy_pcc(window=3, dbeta0=0.01, dbeta_min=0.0025, halve_every=4, target=0.636508)
    g = Group(2 * 10 ** 9, 4, pcc)
    reqs = [(128, 0xA1, 0), (64, 0xA2, 1), (256, 0xA3, 2)]  # (L, seed, admitted at round)
    slot_of, done = {}, {}
    r = 0
    while len(done) < len(reqs):
        for k, (L, seed, adm) in enumerate(reqs):
            if adm == r and k not in slot_of.values():
                slot_of[g.add(L, seed, 1.0, 36, replica=0)] = k
        g.round(4)
        for s in g.poll():
            k = slot_of.pop(s)
            last, beta, bmean = g.result(s)
            done[k] = (beta, g.get_state(s, reqs[k][0]))
            g.release(s)
        r += 1
    g.close()
    for k, (L, seed, adm) in enumerate(reqs):
        orc = oracle.Lattice(L=L, beta=1.0, seed=seed, storage32=True)
        b_o, _ = orc.pcc(12, 3, 0.01, dbeta_min=0.0025, halve_every=4)
        beta, (c, s) = done[k]
        assert beta == b_o[-1], k
        assert np.array_equal(c.astype(np.float64), orc.c) and np.array_equal(s.astype(np.float64), orc.s), k
