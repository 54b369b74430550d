"""The merge inside the labelling tile pass (xy_set_merge_in_pass) against the
CPU oracle directly, on the shapes the schedule-independence test does not
reach: lattices narrower than a 64-column tile (one tile per row band, so a
tile is its own left / upper neighbour), the 64-bit site-index kernels, one
sweep per call (the links-and-labels pass unites the edges), and window-1 PCC
(the window-end pass with both candidates' links, then the labels of the chosen
ones).  Bar as in test_gpu_parity: links, labels and spins bit-exact, the
observables within 1e-10 per site, the PCC beta trace bit-exact.
"""
import numpy as np
import pytest

import oracle
import xyworkloads as wl

pytestmark = pytest.mark.gpu

OBS_TOL = 1e-10
NAMES = ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2")


def _in_pass(lat):
    lat.set_merge(2, 1)
    lat.set_merge_in_pass(True)
    return lat


def _pair(L, seed, tile_rows=0, bits=0, beta=1.12):
    import paper_1210_6116_amd as xy
    lat = _in_pass(xy.Lattices(dict(L=L, beta=beta, seed=seed, tile_rows=tile_rows, label_bits=bits)))
    c0, s0 = wl.random_spins(L, 3 + L)
    lat.set_state(c0, s0)
    orc = oracle.Lattice(L=L, beta=beta, seed=seed, storage32=True, c=c0.astype(np.float64),
                         s=s0.astype(np.float64))
    return lat, orc


@pytest.mark.parametrize("L,tile_rows,bits,wide", [(8, 0, 0, False), (32, 0, 0, False), (64, 32, 0, False),
                                                    (256, 16, 0, False), (256, 64, 0, False), (128, 32, 64, False),
                                                    (128, 32, 64, True), (32, 0, 64, True)])
def test_in_pass_fused_sweeps_match_oracle(L, tile_rows, bits, wide, monkeypatch):
    if wide:
        monkeypatch.setenv("XY_WIDE_INDEX", "1")
    print("in-pass fused L=%d rows=%d bits=%d wide=%d" % (L, tile_rows, bits, wide), flush=True)
    lat, orc = _pair(L, 0x1A9A + L, tile_rows, bits)
    tr_g = lat.sweep(16, trace=True)
    tr_o, ties_o = orc.run(15)
    obs_o, t_o, bx_o, by_o, lab_o = orc.sweep_detail()
    cg, sg = lat.get_state()
    assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s)
    assert np.array_equal(lat.labels(), lab_o)
    bx_g, by_g = lat.bonds()
    assert np.array_equal(bx_g, bx_o) and np.array_equal(by_g, by_o)
    for k, name in enumerate(NAMES):
        assert np.max(np.abs(tr_g[:15, 0][name] - tr_o[:, k])) <= OBS_TOL, name
        assert abs(float(tr_g[15, 0][name]) - obs_o[k]) <= OBS_TOL, name
    lat.close()


@pytest.mark.parametrize("L", [16, 64])
def test_in_pass_single_sweeps_match_oracle(L):
    # one sweep per call: the links-and-labels pass unites the edges, the
    # edge coins run both finalisation stages
    print("in-pass single sweeps L=%d" % L, flush=True)
    lat, orc = _pair(L, 0x51D6 + L)
    for k in range(6):
        tr = lat.sweep(1, trace=True)
        obs_o, ties_o, bx_o, by_o, lab_o = orc.sweep_detail()
        bx_g, by_g = lat.bonds()
        assert np.array_equal(bx_g, bx_o) and np.array_equal(by_g, by_o), k
        assert np.array_equal(lat.labels(), lab_o), k
        cg, sg = lat.get_state()
        assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s), k
        assert int(tr[0, 0]["near_ties"]) == ties_o
        for j, name in enumerate(NAMES):
            assert abs(float(tr[0, 0][name]) - obs_o[j]) <= OBS_TOL, (k, name)
    lat.close()


@pytest.mark.parametrize("L,wide", [(16, False), (64, False), (64, True)])
def test_in_pass_window1_pcc_matches_oracle(L, wide, monkeypatch):
    # window 1: every sweep ends a window, so the flip activates both
    # candidates' links and the next sweep labels the chosen ones, uniting the
    # tile edges in that pass
    if wide:
        monkeypatch.setenv("XY_WIDE_INDEX", "1")
    import paper_1210_6116_amd as xy
    print("in-pass window-1 PCC L=%d wide=%d" % (L, wide), flush=True)
    seed = 0xACE + L
    lat = _in_pass(xy.Lattices(dict(L=L, beta=1.0, seed=seed, label_bits=64 if wide else 0)))
    orc = oracle.Lattice(L=L, beta=1.0, seed=seed, storage32=True)
    means = lat.pcc(24, 1, 0.01, dbeta_min=0.001, halve_every=8, means=True)
    b_o, bu_o = orc.pcc(24, 1, 0.01, dbeta_min=0.001, halve_every=8)
    assert np.array_equal(means[:, 0]["beta"], b_o)
    assert lat.beta() == orc.beta
    cg, sg = lat.get_state()
    assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s)
    lat.close()
