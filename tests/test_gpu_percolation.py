"""The percolation PCC rule on the GPU (through the C ABI) against the oracle.

The wrapping check decides an integer per sweep (does some cluster wind
around the periodic lattice along x, along y?), so its bits must equal the
oracle's (unwrapped-coordinate BFS) bit for bit, and with them the beta trace
of the rule: the kernels take every decision of the sweep exactly as the
oracle does (links, labels, coins and reflections are bit-exact, see
test_gpu_parity.py), and beta moves by +-dbeta from the window's wrapping
fraction, an exact rational.  Cases: window 1 (one sweep per step: the bits
of every sweep), windows of several sweeps (the fused path inside a window),
tile heights 16 / 32 / 64 and lattices narrower than a tile (the seam inside
one tile), a batch of replicas of different sizes, and beta ranges where
wrapping is rare, common and nearly certain.  Bit 8 (the check did not
settle) must never appear.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

WRAP_BITS = 3
CHECKED = 4
UNSETTLED = 8


def _xy():
    import paper_1210_6116_amd as xy
    return xy


def _run_pair(specs, nsteps, window, dbeta0, dbeta_min=0.0, halve_every=0, target=0.5):
    """The same percolation PCC run on one GPU handle (all specs as replicas)
    and on the oracle, replica by replica; returns both sides' records."""
    xy = _xy()
    print("percolation PCC %s steps=%d window=%d" % ([(s["L"], s["beta"], s.get("tile_rows", 0)) for s in specs],
                                                     nsteps, window), flush=True)
    lat = xy.Lattices(specs)
    means = lat.pcc(nsteps, window, dbeta0, dbeta_min=dbeta_min, halve_every=halve_every, target=target,
                    means=True, rule=xy.XY_PCC_PERCOLATION)
    betas = [lat.beta(k) for k in range(len(specs))]
    lat.close()
    out = []
    for k, sp in enumerate(specs):
        orc = oracle.Lattice(L=sp["L"], beta=sp["beta"], seed=sp["seed"], rep=sp.get("rep", 0), storage32=True)
        b_o, p_o, w_o = orc.pcc_perc(nsteps, window, dbeta0, dbeta_min=dbeta_min, halve_every=halve_every,
                                     target=target)
        out.append((means[:, k], betas[k], b_o, p_o, w_o.reshape(nsteps, window)))
    return out


@pytest.mark.parametrize("L,rows,beta", [(4, 0, 1.1), (8, 0, 0.9), (16, 16, 1.0), (32, 16, 1.05),
                                         (64, 32, 1.1), (128, 16, 1.12), (128, 64, 1.0), (256, 32, 1.12)])
def test_wrap_bits_every_sweep(L, rows, beta):
    """Window 1: each step is one sweep, its window mean that sweep's bits."""
    spec = dict(L=L, beta=beta, seed=0x5EA7 + L, rep=L % 5, tile_rows=rows)
    n = 60 if L <= 128 else 30
    (m, beta_end, b_o, p_o, w_o), = _run_pair([spec], n, 1, 0.01, dbeta_min=0.0025, halve_every=10)
    wrap_g = m["wrap"].astype(np.int64)
    assert np.all(wrap_g & CHECKED) and not np.any(wrap_g & UNSETTLED)
    assert np.array_equal(wrap_g & WRAP_BITS, w_o[:, 0]), (np.flatnonzero((wrap_g & WRAP_BITS) != w_o[:, 0])[:5])
    assert np.array_equal(m["perc"], p_o)
    assert np.array_equal(m["beta"], b_o)
    assert beta_end == b_o[-1]
    # the run visits both outcomes (otherwise the parity says little)
    assert 0 < np.count_nonzero(w_o) < n, w_o[:, 0]


def test_windows_and_batch():
    """Windows of 7 sweeps (the fused pass inside a window) over a batch of
    replicas of different sizes and tile shapes; the window fraction and the
    union of the window's bits per replica."""
    specs = [dict(L=L, beta=b, seed=0xBEE + k, rep=k, tile_rows=rows)
             for k, (L, b, rows) in enumerate(((64, 0.95, 32), (32, 1.15, 16), (128, 1.05, 32), (16, 1.3, 16)))]
    for m, beta_end, b_o, p_o, w_o in _run_pair(specs, 12, 7, 0.02, dbeta_min=0.005, halve_every=4):
        assert np.array_equal(m["perc"], p_o)
        union = np.bitwise_or.reduce(w_o, axis=1)
        assert np.array_equal(m["wrap"].astype(np.int64), union | CHECKED)
        assert np.array_equal(m["beta"], b_o)
        assert beta_end == b_o[-1]


def test_extremes():
    """beta = 0: no links, nothing winds, beta rises every step; beta = 4 from
    a thermalised start: clusters wind in most sweeps, beta falls every step."""
    xy = _xy()
    lat = xy.Lattices(dict(L=64, beta=0.0, seed=5))
    m = lat.pcc(5, 3, 0.01, means=True, rule=xy.XY_PCC_PERCOLATION, target=0.5)
    assert np.all(m["perc"][:, 0] == 0.0) and np.all(m["wrap"][:, 0] == CHECKED)
    assert np.allclose(m["beta"][:, 0], 0.01 * np.arange(1, 6))
    lat.close()
    lat = xy.Lattices(dict(L=64, beta=4.0, seed=6))
    lat.sweep(50)
    m = lat.pcc(5, 3, 0.01, means=True, rule=xy.XY_PCC_PERCOLATION, target=0.5)
    assert np.all(m["perc"][:, 0] >= 0.5) and np.all(m["wrap"][:, 0] & CHECKED)
    assert np.allclose(m["beta"][:, 0], 4.0 - 0.01 * np.arange(1, 6))
    lat.close()


def test_helicity_runs_report_no_wrapping_check():
    xy = _xy()
    lat = xy.Lattices(dict(L=32, beta=1.1, seed=7))
    m = lat.pcc(3, 2, 0.01, means=True)
    assert np.all(m["wrap"] == 0) and np.all(m["perc"] == -1.0)
    tr = lat.sweep(3, trace=True)
    assert np.all(tr["wrap"] == 0) and np.all(tr["perc"] == -1.0)
    lat.close()


def test_rule_errors():
    xy = _xy()
    from paper_1210_6116_amd import _lib
    lat = xy.Lattices(dict(L=8192, beta=1.1, seed=8))
    with pytest.raises(_lib.XYError) as ei:
        lat.pcc(1, 1, 0.01, rule=xy.XY_PCC_PERCOLATION)
    assert ei.value.code == _lib.XY_EINVAL
    with pytest.raises(_lib.XYError) as ei:
        lat.pcc(1, 1, 0.01, rule=7)
    assert ei.value.code == _lib.XY_EINVAL
    assert lat.sweep_count()[0] == 0  # nothing ran
    lat.close()
    from paper_1210_6116_amd.serve import Group
    with pytest.raises(_lib.XYError) as ei:
        Group(2 * 10 ** 9, 4, xy.xy_pcc(window=1, dbeta0=0.01, dbeta_min=0.0, halve_every=0, target=0.5,
                                         rule=xy.XY_PCC_PERCOLATION))
    assert ei.value.code == _lib.XY_EINVAL
