"""Autotuner (paper_1210_6116_amd.autotune): tile height and merge schedule.

The tuner times each candidate tile height on the replica set and keeps the
fastest; the choice only changes speed, never results: links, labels and coins
are functions of the lattice, the sweep and the canonical roots, not of the
tiling.  Checks: the pick is a candidate with the smallest measured time, the
cache round-trips it, and replicas swept with every candidate height end in
bit-identical states and observables.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _specs():
    return [dict(L=L, beta=b, seed=0xA070 + k, rep=k)
            for k, (L, b) in enumerate([(64, 1.0), (128, 1.12), (256, 1.05), (64, 1.2), (512, 1.1)])]


def test_autotune_pick_and_cache(tmp_path, monkeypatch):
    from paper_1210_6116_amd import autotune
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    specs = _specs()
    best, timings = autotune.tune(specs, sweeps=5, warmup=2, use_cache=False)
    print("autotune:", best, {k: "%.1f us" % (v * 1e6) for k, v in timings.items()}, flush=True)
    assert set(timings) == set(autotune.CANDIDATES)
    assert best in autotune.CANDIDATES and timings[best] == min(timings.values())
    assert all(v > 0 for v in timings.values())
    # the cached record gives the same pick without timing again
    again, cached = autotune.tune(specs, use_cache=True)
    assert again == best
    assert cached == pytest.approx(timings)
    assert autotune.tile_rows(specs) == best


def test_results_do_not_depend_on_tile_height():
    import paper_1210_6116_amd as xy
    from paper_1210_6116_amd import autotune
    specs = _specs()
    runs = {}
    for rows in autotune.CANDIDATES:
        lat = xy.Lattices([dict(s, tile_rows=rows) for s in specs])
        tr = lat.sweep(12, trace=True)
        states = [lat.get_state(k) for k in range(len(specs))]
        lat.close()
        runs[rows] = (tr, states)
    ref_tr, ref_states = runs[autotune.CANDIDATES[0]]
    for rows, (tr, states) in runs.items():
        for f in ("E", "m2", "ex", "sx", "mk2"):
            np.testing.assert_allclose(tr[f], ref_tr[f], rtol=1e-10, atol=1e-12, err_msg="%s rows=%d" % (f, rows))
        for k in range(len(specs)):
            assert np.array_equal(states[k][0], ref_states[k][0]), (rows, k)
            assert np.array_equal(states[k][1], ref_states[k][1]), (rows, k)


def test_merge_schedule_pick_and_cache(tmp_path, monkeypatch):
    """One L = 2048 lattice: every merge schedule is timed, the pick is the
    fastest, and the cache returns it."""
    from paper_1210_6116_amd import autotune
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    specs = [dict(L=2048, beta=1.12, seed=0xB0B)]
    best, timings = autotune.tune_merge(specs, 32, sweeps=8, warmup=2, use_cache=False)
    print("merge schedule:", best, {k: "%.1f us" % (v * 1e6) for k, v in timings.items()}, flush=True)
    assert set(timings) == set(autotune.merge_candidates())
    assert timings[best] == min(timings.values())
    again, cached = autotune.tune_merge(specs, 32, use_cache=True)
    assert again == best and cached == pytest.approx(timings)


@pytest.mark.parametrize("beta", [0.5, 1.12])
def test_results_do_not_depend_on_merge_schedule(beta):
    """Every (dedup, edges per wave) choice: bit-identical traces, spins and
    labels, for a replica batch (graph replay included) and one lattice."""
    import paper_1210_6116_amd as xy
    from paper_1210_6116_amd import autotune
    specs = [dict(L=1024, beta=beta, seed=0xD0D)] + [dict(L=L, beta=beta, seed=0xD0E + k, rep=k)
                                                    for k, L in enumerate((64, 256, 128))]
    runs = {}
    for choice in autotune.merge_candidates():
        lat = xy.Lattices(specs)
        autotune.configure(lat, choice)
        tr = lat.sweep(7, trace=True)
        lat.sweep_graph(3, 2)
        tr2 = lat.sweep(1, trace=True)
        runs[choice] = (tr, tr2, [lat.get_state(k) for k in range(len(specs))],
                        [lat.labels(k) for k in range(len(specs))])
        lat.close()
    ref = runs[autotune.merge_candidates()[0]]
    for choice, (tr, tr2, st, lab) in runs.items():
        for f in ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2", "near_ties"):
            assert np.array_equal(tr[f], ref[0][f]) and np.array_equal(tr2[f], ref[1][f]), (choice, f)
        for k in range(len(specs)):
            assert np.array_equal(st[k][0], ref[2][k][0]) and np.array_equal(st[k][1], ref[2][k][1]), (choice, k)
            assert np.array_equal(lab[k], ref[3][k]), (choice, k)


def test_merge_schedule_tuned_on_a_pcc_call(tmp_path, monkeypatch):
    """tune_merge timing the workload's own call (window-1 PCC, whose window
    ends run the two-candidate and chosen-labels passes): every choice timed,
    the pick cached under its tag apart from the plain-sweep record, and every
    choice gives the same beta trace and state."""
    import paper_1210_6116_amd as xy
    from paper_1210_6116_amd import autotune
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    spec = dict(L=256, beta=1.0, seed=0xCAFE)

    def pcc_step(lat, n):
        lat.pcc(n, 1, 0.004, dbeta_min=0.0005, halve_every=50)

    best, timings = autotune.tune_merge([spec], 32, sweeps=4, warmup=4, repeats=1, use_cache=False,
                                        step=pcc_step, tag="pcc-w1")
    print("pcc merge schedule:", best, flush=True)
    assert set(timings) == set(autotune.merge_candidates()) and timings[best] == min(timings.values())
    again, cached = autotune.tune_merge([spec], 32, step=pcc_step, tag="pcc-w1")
    assert again == best and cached == pytest.approx(timings)
    runs = {}
    for choice in autotune.merge_candidates():
        lat = xy.Lattices(spec)
        autotune.configure(lat, choice)
        means = lat.pcc(30, 1, 0.004, dbeta_min=0.0005, halve_every=50, means=True)
        runs[choice] = (means[:, 0]["beta"].copy(), lat.get_state())
        lat.close()
    ref_beta, (ref_c, ref_s) = runs[autotune.merge_candidates()[0]]
    for choice, (beta, (c, s)) in runs.items():
        assert np.array_equal(beta, ref_beta), choice
        assert np.array_equal(c, ref_c) and np.array_equal(s, ref_s), choice
