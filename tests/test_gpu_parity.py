"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Same seeded inputs on both sides (random FP32 states from xyworkloads, or each
side's own Philox hot start).  Bar:
  * bit planes of active links, canonical labels, mirror directions, hot start:
    bit-exact (integer / index results, and FP64 values both sides obtain with
    correctly rounded operations only);
  * spins: the benchmark spec's bound is 1e-6 absolute; the kernels round the same FP64
    expressions once to FP32, so they are required here to be bit-identical;
  * observables (FP64 sums in a different order): 1e-10 absolute per site.
A near tie (|u - p| < 1e-9) could legitimately flip a link decision between two
correct implementations; ties are counted on both sides and must agree.
"""
import numpy as np
import pytest

import oracle
import xyworkloads as wl

pytestmark = pytest.mark.gpu

OBS_TOL = 1e-10
NAMES = ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2")


def _gpu():
    import paper_1210_6116_amd as xy
    return xy


def _check_obs(g, o, where):
    for k, name in enumerate(NAMES):
        assert abs(float(g[name]) - o[k]) <= OBS_TOL, (where, name, float(g[name]), o[k])


def _trajectory(L, beta, seed, rep=0, nsweeps=10, tile_rows=0, label_bits=0, state_seed=None):
    xy = _gpu()
    print("trajectory L=%d beta=%g tile_rows=%d label_bits=%d" % (L, beta, tile_rows, label_bits), flush=True)
    lat = xy.Lattices(dict(L=L, beta=beta, seed=seed, rep=rep, tile_rows=tile_rows, label_bits=label_bits))
    if state_seed is not None:
        c0, s0 = wl.random_spins(L, state_seed)
        lat.set_state(c0, s0)
        orc = oracle.Lattice(L=L, beta=beta, seed=seed, rep=rep, storage32=True,
                             c=c0.astype(np.float64), s=s0.astype(np.float64))
    else:
        orc = oracle.Lattice(L=L, beta=beta, seed=seed, rep=rep, storage32=True)
        cg, sg = lat.get_state()
        assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s)
    for k in range(nsweeps):
        t, r = lat.sweep_count()
        assert t == k
        assert np.array_equal(r, oracle.direction(seed, rep, k)), (k, r)
        tr = lat.sweep(1, trace=True)
        obs_o, ties_o, bx_o, by_o, lab_o = orc.sweep_detail()
        bx_g, by_g = lat.bonds()
        assert int(tr[0, 0]["near_ties"]) == ties_o
        assert np.array_equal(bx_g, bx_o), ("bx", k, np.flatnonzero(bx_g != bx_o)[:10])
        assert np.array_equal(by_g, by_o), ("by", k, np.flatnonzero(by_g != by_o)[:10])
        lab_g = lat.labels()
        assert np.array_equal(lab_g, lab_o), ("labels", k, np.flatnonzero(lab_g != lab_o)[:10])
        cg, sg = lat.get_state()
        assert np.array_equal(cg.astype(np.float64), orc.c), ("cos", k, np.max(np.abs(cg - orc.c)))
        assert np.array_equal(sg.astype(np.float64), orc.s), ("sin", k, np.max(np.abs(sg - orc.s)))
        _check_obs(tr[0, 0], obs_o, ("sweep", k))
        assert int(tr[0, 0]["sweep"]) == k + 1
    lat.close()


def test_hot_start_and_directions_bit_exact():
    for L, seed, rep in ((2, 3, 0), (8, 0x12106116, 1), (64, 0x12106116, 0), (256, 99, 5)):
        _trajectory(L, 1.12, seed, rep=rep, nsweeps=2)


@pytest.mark.parametrize("L,tile_rows", [(2, 0), (4, 0), (8, 0), (16, 0), (32, 16), (64, 16), (64, 32),
                                         (64, 64), (128, 16), (256, 32), (512, 64)])
def test_trajectory_parity(L, tile_rows):
    _trajectory(L, 1.12, 0x12106116 + L, rep=L % 7, nsweeps=10, tile_rows=tile_rows, state_seed=1000 + L)


@pytest.mark.parametrize("L", [8, 64, 256])
def test_trajectory_parity_uint64_labels(L):
    _trajectory(L, 1.12, 0x600D + L, nsweeps=6, label_bits=64, state_seed=77 + L)


@pytest.mark.parametrize("beta", [0.0, 0.3, 2.5, 10.0])
def test_trajectory_parity_other_beta(beta):
    _trajectory(64, beta, 0xBE7A, nsweeps=4, tile_rows=32, state_seed=5)


def test_beta_zero_labels_identity():
    xy = _gpu()
    lat = xy.Lattices(dict(L=128, beta=0.0, seed=1))
    lat.sweep(3)
    assert np.array_equal(lat.labels(), np.arange(128 * 128))
    bx, by = lat.bonds()
    assert bx.sum() == 0 and by.sum() == 0
    lat.close()


def test_renormalisation_sweep_parity():
    # crosses sweep 1023, after which every spin is rescaled to unit length
    xy = _gpu()
    L, beta, seed = 16, 1.12, 4321
    lat = xy.Lattices(dict(L=L, beta=beta, seed=seed))
    orc = oracle.Lattice(L=L, beta=beta, seed=seed, storage32=True)
    tr_g = lat.sweep(1030, trace=True)
    tr_o, ties_o = orc.run(1030)
    cg, sg = lat.get_state()
    assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s)
    for k, name in enumerate(NAMES):
        assert np.max(np.abs(tr_g[:, 0][name] - tr_o[:, k])) <= OBS_TOL, name
    assert np.array_equal(tr_g[:, 0]["near_ties"].astype(np.int64), ties_o)
    lat.close()


def test_measure_matches_oracle():
    xy = _gpu()
    for L in (2, 16, 64, 256):
        lat = xy.Lattices(dict(L=L, beta=0.9, seed=L))
        c, s = wl.random_spins(L, 31 + L)
        lat.set_state(c, s)
        g = lat.measure()[0]
        _check_obs(g, oracle.measure(L, c.astype(np.float64), s.astype(np.float64), 0.9), ("measure", L))
        lat.close()


@pytest.mark.parametrize("L,tile_rows,bits", [(8, 0, 32), (64, 16, 32), (128, 32, 64), (256, 64, 32),
                                              (256, 16, 64)])
def test_label_links_patterns_and_random(L, tile_rows, bits):
    xy = _gpu()
    cases = [(k, wl.pattern_bonds(L, k)) for k in wl.PATTERNS]
    cases += [("rand%.1f" % p, wl.random_bonds(L, p, 11 + int(10 * p))) for p in (0.2, 0.5, 0.6, 0.8)]
    for name, (bx, by) in cases:
        print("label_links L=%d rows=%d bits=%d %s" % (L, tile_rows, bits, name), flush=True)
        got = xy.label_links(L, bx, by, label_bits=bits, tile_rows=tile_rows)
        assert np.array_equal(got, oracle.label(L, bx, by)), name


def test_pcc_parity_small():
    xy = _gpu()
    L, seed = 16, 0xACC
    lat = xy.Lattices(dict(L=L, beta=1.0, seed=seed))
    orc = oracle.Lattice(L=L, beta=1.0, seed=seed, storage32=True)
    means = lat.pcc(12, 3, 0.01, dbeta_min=0.001, halve_every=4, means=True)
    b_o, bu_o = orc.pcc(12, 3, 0.01, dbeta_min=0.001, halve_every=4)
    assert np.array_equal(means[:, 0]["beta"], b_o)
    assert lat.beta() == orc.beta
    cg, sg = lat.get_state()
    assert np.array_equal(cg.astype(np.float64), orc.c)
    lat.close()


def test_batched_replicas_match_plain():
    xy = _gpu()
    specs = [dict(L=L, beta=b, seed=0xBA7C, rep=k) for k, (L, b) in
             enumerate([(64, 1.0), (128, 1.1), (16, 1.2), (256, 1.05), (64, 1.15)])]
    batch = xy.Lattices(specs)
    tb = batch.sweep(5, trace=True)
    for k, spec in enumerate(specs):
        one = xy.Lattices(spec)
        t1 = one.sweep(5, trace=True)
        c1, s1 = one.get_state()
        cb, sb = batch.get_state(k)
        assert np.array_equal(c1, cb) and np.array_equal(s1, sb), k
        assert np.array_equal(one.labels(), batch.labels(k)), k
        for name in NAMES:
            assert np.array_equal(t1[:, 0][name], tb[:, k][name]), (k, name)
        one.close()
    batch.close()


def test_batched_512_replicas_sampled_against_oracle():
    # The batched workload at its full shape (512 replicas, L = 64 ... 2048, beta in
    # [1.0, 1.2], 64-row tiles, the merge schedule the bench's tuner picks for it:
    # hash deduplication, 4 tile edges per merge wave; sweeps replayed from a
    # captured graph): two replicas of every size, L = 64 ... 2048, are checked
    # against the oracle bit for bit (the L = 512 ... 2048 replicas carry most of
    # the batch's work)
    xy = _gpu()
    specs = [dict(sp, tile_rows=64) for sp in wl.batched_replicas(512)]
    picks = []
    for L in (64, 128, 256, 512, 1024, 2048):
        picks += [k for k, sp in enumerate(specs) if sp["L"] == L][:2]
    assert len(picks) == 12
    print("512-replica batch, sampled replicas %s" % picks, flush=True)
    batch = xy.Lattices(specs)
    batch.set_merge(2, 4)
    nsw = 3
    batch.sweep_graph(nsw, 1)
    meas = batch.measure()
    for k in picks:
        sp = specs[k]
        print("replica %d: L=%d beta=%.4f" % (k, sp["L"], sp["beta"]), flush=True)
        orc = oracle.Lattice(L=sp["L"], beta=sp["beta"], seed=sp["seed"], rep=sp["rep"], storage32=True)
        for _ in range(nsw):
            obs_o, _, _, _, lab_o = orc.sweep_detail()
        c, s = batch.get_state(k)
        assert np.array_equal(c.astype(np.float64), orc.c) and np.array_equal(s.astype(np.float64), orc.s), k
        assert np.array_equal(batch.labels(k), lab_o), k
        _check_obs(meas[k], obs_o, ("replica", k))
        assert batch.sweep_count(k)[0] == nsw
    # every replica: unit spins and the same sweep count
    for k in range(0, 512, 37):
        c, s = batch.get_state(k)
        n2 = c.astype(np.float64) ** 2 + s.astype(np.float64) ** 2
        assert np.max(np.abs(n2 - 1.0)) < 1e-6, k
        assert batch.sweep_count(k)[0] == nsw
    batch.close()


def test_full_size_l4096_one_sweep():
    # The bench configuration (L = 4096, beta = 1.12, default tiles): one sweep
    # checked element by element against the oracle.
    _trajectory(4096, 1.12, wl.SEED_L4096, nsweeps=1, state_seed=4096)


@pytest.mark.parametrize("L,tile_rows,bits", [(8, 0, 0), (64, 32, 0), (256, 16, 0), (256, 64, 0), (128, 32, 64)])
def test_fused_multi_sweep_parity(L, tile_rows, bits):
    # one call of many sweeps: every sweep but the last runs the fused
    # flip(t) + links(t+1) pass
    xy = _gpu()
    print("fused L=%d rows=%d bits=%d" % (L, tile_rows, bits), flush=True)
    seed = 0xF05E + L
    lat = xy.Lattices(dict(L=L, beta=1.12, seed=seed, tile_rows=tile_rows, label_bits=bits))
    c0, s0 = wl.random_spins(L, 9 + L)
    lat.set_state(c0, s0)
    orc = oracle.Lattice(L=L, beta=1.12, seed=seed, storage32=True, c=c0.astype(np.float64),
                         s=s0.astype(np.float64))
    tr_g = lat.sweep(20, trace=True)
    tr_o, ties_o = orc.run(19)
    obs_o, t_o, bx_o, by_o, lab_o = orc.sweep_detail()
    cg, sg = lat.get_state()
    assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s)
    assert np.array_equal(lat.labels(), lab_o)
    bx_g, by_g = lat.bonds()
    assert np.array_equal(bx_g, bx_o) and np.array_equal(by_g, by_o)
    for k, name in enumerate(NAMES):
        assert np.max(np.abs(tr_g[:19, 0][name] - tr_o[:, k])) <= OBS_TOL, name
        assert abs(float(tr_g[19, 0][name]) - obs_o[k]) <= OBS_TOL, name
    lat.close()


@pytest.mark.parametrize("L", [64, 2048])
def test_fused_and_single_sweeps_identical(L):
    # the fused pass (deferred finalisation in the merge and edge-coin
    # kernels) and one sweep per call (flip, then k_finalize) sum the same
    # tile partials with the same two-stage arithmetic: identical traces
    xy = _gpu()
    print("fused vs single L=%d" % L, flush=True)
    spec = dict(L=L, beta=1.12, seed=0x5EED + L)
    a = xy.Lattices(spec)
    b = xy.Lattices(spec)
    tr_a = a.sweep(12, trace=True)
    tr_b = np.concatenate([b.sweep(1, trace=True) for _ in range(12)])
    assert tr_a.shape == tr_b.shape
    for name in NAMES + ("near_ties", "sweep"):
        assert np.array_equal(tr_a[:, 0][name], tr_b[:, 0][name]), name
    ca, sa = a.get_state()
    cb, sb = b.get_state()
    assert np.array_equal(ca, cb) and np.array_equal(sa, sb)
    a.close()
    b.close()


@pytest.mark.parametrize("L,nsweeps", [(64, 6), (256, 4)])
def test_wide_index_path_parity(L, nsweeps, monkeypatch):
    # the 64-bit site-index kernels that lattices above 2^30 sites use
    monkeypatch.setenv("XY_WIDE_INDEX", "1")
    _trajectory(L, 1.12, 0x91DE + L, nsweeps=nsweeps, label_bits=64, state_seed=5 + L)


def test_wide_index_fused_parity(monkeypatch):
    monkeypatch.setenv("XY_WIDE_INDEX", "1")
    test_fused_multi_sweep_parity(128, 32, 64)


def test_device_label_flatten_and_views():
    # canonical labels written to caller-owned device memory in both widths,
    # and the device views of the state and link planes, against the host copies
    import torch
    xy = _gpu()
    L = 128
    lat = xy.Lattices(dict(L=L, beta=1.12, seed=0xF1A7))
    lat.sweep(3)
    want = lat.labels()
    assert np.array_equal(lat.labels_device(bits=64).cpu().numpy(), want)
    assert np.array_equal(lat.labels_device(bits=32).cpu().numpy().view(np.uint32).astype(np.int64), want)
    v = lat.views()
    c, s = lat.get_state()
    assert np.array_equal(v["cos"].cpu().numpy(), c) and np.array_equal(v["sin"].cpu().numpy(), s)
    bx, by = lat.bonds()
    assert np.array_equal(xy.unpack_bits(v["bx"].cpu().numpy().view(np.uint32), L * L), bx)
    assert np.array_equal(xy.unpack_bits(v["by"].cpu().numpy().view(np.uint32), L * L), by)
    assert v["sweep"] == 3 and v["L"] == L
    torch.cuda.synchronize()
    lat.close()
