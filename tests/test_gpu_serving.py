"""Batched graph replay and the serving group, through the C ABI.

Tolerance for every comparison here is 0: replicas never interact (tiles belong
to one replica, sums are per replica in a fixed order, random numbers are keyed
by the replica's own seed and stream id), so a request's trajectory is the same
bit for bit alone, in a batch, or in a served mix.
"""
import numpy as np
import pytest

import xyworkloads as wl

pytestmark = pytest.mark.gpu

NAMES = ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2")


def test_graph_replay_equals_sweeps():
    """Every replay of a captured 10-sweep graph equals 10 eager sweeps; eager
    work (a measurement, host reads) and synchronisations run between the
    replays, and the last replay's results are checked like the first's."""
    import paper_1210_6116_amd as xy
    specs = [dict(L=L, beta=1.1, seed=0x6A, rep=k) for k, L in enumerate((64, 256, 128))]
    a = xy.Lattices(specs)
    b = xy.Lattices(specs)
    for replay in range(4):
        a.sweep(10)
        b.sweep_graph(10, 1)
        for k in range(len(specs)):
            ca, sa = a.get_state(k)
            cb, sb = b.get_state(k)
            assert np.array_equal(ca, cb) and np.array_equal(sa, sb), (replay, k)
            assert np.array_equal(a.labels(k), b.labels(k)), (replay, k)
            assert a.sweep_count(k)[0] == b.sweep_count(k)[0] == 10 * (replay + 1)
        ma, mb = a.measure(), b.measure()
        for name in NAMES:
            assert np.array_equal(ma[name], mb[name]), (replay, name)
    # several replays in one call
    a.sweep(30)
    b.sweep_graph(10, 3)
    for k in range(len(specs)):
        assert np.array_equal(a.get_state(k)[0], b.get_state(k)[0])
        assert np.array_equal(a.labels(k), b.labels(k))
    a.close()
    b.close()


def _pcc():
    from paper_1210_6116_amd import xy_pcc
    return xy_pcc(window=1, dbeta0=0.004, dbeta_min=0.0005, halve_every=25, target=0.636508)


def _run_group(requests, budget=2 * 10 ** 9, max_slots=8, rounds=7):
    """requests: list of (admit_round, L, seed, sweeps). Returns {index: result}."""
    from paper_1210_6116_amd.serve import Group
    g = Group(budget, max_slots, _pcc())
    out, slot_of = {}, {}
    r = 0
    while len(out) < len(requests):
        for k, (adm, L, seed, sweeps) in enumerate(requests):
            if adm == r and k not in slot_of.values():
                # a request's stream is (seed, replica 0) whatever its position in the mix
                s = g.add(L, seed, 1.0, sweeps, replica=0)
                assert s is not None
                slot_of[s] = k
        g.round(rounds)
        for s in g.poll():
            out[slot_of.pop(s)] = g.result(s)
            g.release(s)
        r += 1
    g.close()
    return out


def test_served_result_same_alone_and_in_mix():
    target = (0, 256, 0xA11CE, 40)
    alone = _run_group([target])[0]
    mix = _run_group([(0, 512, 7, 25), (1, 128, 8, 60), target, (2, 64, 9, 33), (3, 256, 10, 11)])[2]
    for name in NAMES:
        assert alone[0][name] == mix[0][name], name
    assert alone[1] == mix[1] and alone[2] == mix[2]
    assert int(alone[0]["sweep"]) == int(mix[0]["sweep"]) == 40


def test_served_result_equals_plain_pcc_run():
    import paper_1210_6116_amd as xy
    L, seed, sweeps = 128, 0xBEE, 30
    served = _run_group([(0, L, seed, sweeps)])[0]
    lat = xy.Lattices(dict(L=L, beta=1.0, seed=seed, rep=0))
    means = lat.pcc(sweeps, 1, 0.004, dbeta_min=0.0005, halve_every=25, means=True)
    assert lat.beta() == served[1]
    assert np.mean(means[:, 0]["beta"]) == pytest.approx(served[2], abs=1e-12)
    lat.close()


def test_served_request_matches_oracle():
    """One served request (L = 128, window-1 PCC with the halving schedule) in a
    mix that changes around it, against the oracle's PCC run: the beta after
    every sweep and the final spins bit for bit."""
    import oracle
    from paper_1210_6116_amd.serve import Group
    L, seed, rep, sweeps = 128, 0x5E12BE, 3, 40
    g = Group(2 * 10 ** 9, 8, _pcc())
    # (round of admission, L, seed, replica, sweeps) of the other requests
    others = [(0, 256, 11, 0, 17), (0, 64, 12, 1, 50), (5, 512, 13, 2, 9), (12, 128, 14, 4, 21), (30, 64, 15, 5, 40)]
    target = g.add(L, seed, 1.0, sweeps, replica=rep)
    assert target is not None
    betas = []
    slots = {}
    for r in range(sweeps):
        for (adm, Lo, so, ro, nso) in others:
            if adm == r:
                s = g.add(Lo, so, 1.0, nso, replica=ro)
                assert s is not None
                slots[s] = (Lo, so)
        assert g.round(1) == 1
        betas.append(g.result(target)[1])
        for s in g.poll():
            if s != target:
                g.release(s)
    c_g, s_g = g.get_state(target, L)
    last, beta, _ = g.result(target)
    g.release(target)
    g.close()
    orc = oracle.Lattice(L=L, beta=1.0, seed=seed, rep=rep, storage32=True)
    btr, _ = orc.pcc(sweeps, 1, 0.004, dbeta_min=0.0005, halve_every=25)
    assert np.array_equal(np.array(betas), btr), np.flatnonzero(np.array(betas) != btr)[:5]
    assert beta == orc.beta
    assert np.array_equal(c_g.astype(np.float64), orc.c) and np.array_equal(s_g.astype(np.float64), orc.s)
    assert int(last["sweep"]) == sweeps


def test_group_budget_and_release():
    from paper_1210_6116_amd import _lib
    from paper_1210_6116_amd.serve import Group
    p = _lib.xy_params(L=256, beta=1.0, seed=1, replica=0, label_bits=0, start=0, tile_rows=0)
    need = _lib.xy_group_bytes(p)
    g = Group(2 * need + need // 2, 8, _pcc())
    s0 = g.add(256, 1, 1.0, 5)
    s1 = g.add(256, 2, 1.0, 5)
    assert s0 is not None and s1 is not None
    assert g.add(256, 3, 1.0, 5) is None          # budget exhausted
    assert g.info() == (2 * need, 2)
    assert g.round(100) == 5
    assert sorted(g.poll()) == sorted([s0, s1])
    g.release(s0)
    assert g.add(256, 3, 1.0, 5) is not None      # memory came back
    # a request larger than the whole budget can never fit: an error, not a wait
    with pytest.raises(_lib.XYError) as ei:
        g.add(1024, 4, 1.0, 5)
    assert ei.value.code == _lib.XY_EINVAL
    g.close()


def test_serve_trace_small():
    from paper_1210_6116_amd.serve import serve
    trace = wl.serving_trace(n_requests=6, rate=50.0, lmin_log2=6, jmax=2, sweeps_lo=10, sweeps_hi=40)
    res = serve(trace, budget_bytes=10 ** 9, max_slots=4, round_sweeps=8)
    s = res["summary"]
    assert s["n"] == 6 and s["served_updates_per_s"] > 0 and s["ttc_p99_s"] >= s["ttc_p50_s"] > 0
    for r in res["requests"]:
        assert r["finished"] >= r["admitted"] >= r["arrival"] - 1e-9
