"""Checks at the full sizes of the timed workloads.

L = 4096 (the plain-sweep throughput lattice): several sweeps in one call run
the fused flip + next-links pass exactly as the throughput run does; the whole
state, the labels, the links and every observable are compared with the oracle
element by element.

L = 65536 (N = 2^32 sites, 64-bit labels; the PCC throughput lattice): the
oracle cannot hold it, so the sweep is checked
  * on a seeded sample of links and sites that the oracle decides one by one:
    link decisions from the pre-sweep spins (bit-exact) and reflections of the
    sampled sites given their cluster roots (bit-exact);
  * everywhere, on the device, by properties of the canonical labels that hold
    at any size: a site's label is no larger than the site and labels itself;
    the two ends of every active link share a label; spins stay unit vectors;
    and the observables equal an FP64 recomputation of the sums from the state.
  * for at least 50 seeded sites whose clusters hold at most 10^5 sites (sites
    in the bottom rows among them, whose cluster keys are near 2^32, the top of
    the 32-bit node and key range of the boundary forest): a breadth-first
    search on the host over the device's link bits, fetched by windows around
    the site, gives exactly the set of sites that carry the site's device label
    (same size as the device count of that label, and its smallest site is the
    label), so no other cluster was united with it and none of it is missing.
"""
import numpy as np
import pytest
import torch

import oracle
import xyworkloads as wl
from clusters import host_cluster

pytestmark = pytest.mark.gpu

OBS_TOL = 1e-10
NAMES = ("E", "m2", "ex", "sx", "ey", "sy", "ups_x", "mk2")


@pytest.mark.parametrize("merge", [(0, 1, 0), (2, 1, 1)])
def test_full_size_l4096_fused_sweeps(merge):
    # the default merge schedule, and the one the bench's tuner picks for this
    # lattice (hash deduplication, the merge inside the labelling pass)
    import paper_1210_6116_amd as xy
    from paper_1210_6116_amd import autotune
    L, beta, seed = 4096, 1.12, wl.SEED_L4096
    print("L=4096 fused sweeps, merge schedule %s" % (merge,), flush=True)
    lat = xy.Lattices(dict(L=L, beta=beta, seed=seed))
    autotune.configure(lat, merge)
    c0, s0 = wl.random_spins(L, 4097)
    lat.set_state(c0, s0)
    orc = oracle.Lattice(L=L, beta=beta, seed=seed, storage32=True, c=c0.astype(np.float64),
                         s=s0.astype(np.float64))
    tr_g = lat.sweep(3, trace=True)
    tr_o, ties_o = orc.run(2)
    obs_o, t_o, bx_o, by_o, lab_o = orc.sweep_detail()
    cg, sg = lat.get_state()
    assert np.array_equal(cg.astype(np.float64), orc.c) and np.array_equal(sg.astype(np.float64), orc.s)
    bx_g, by_g = lat.bonds()
    assert np.array_equal(bx_g, bx_o) and np.array_equal(by_g, by_o)
    assert np.array_equal(lat.labels(), lab_o)
    for k, name in enumerate(NAMES):
        assert np.max(np.abs(tr_g[:2, 0][name] - tr_o[:, k])) <= OBS_TOL, name
        assert abs(float(tr_g[2, 0][name]) - obs_o[k]) <= OBS_TOL, name
    assert int(tr_g[2, 0]["near_ties"]) == t_o
    lat.close()


def _bits(words: torch.Tensor, lo: int, n: int) -> torch.Tensor:
    """Bits lo .. lo+n-1 of a little-endian int32 word plane (lo, n multiples of 32)."""
    w = words[lo // 32:(lo + n) // 32]
    sh = torch.arange(32, device=w.device, dtype=torch.int32)
    return ((w.unsqueeze(1) >> sh) & 1).reshape(-1).bool()


def test_l65536_sampled_oracle_and_invariants():
    import paper_1210_6116_amd as xy
    L, beta, seed, rep = 65536, 1.12, wl.SEED_L65536, 0
    N = L * L
    print("L=65536 allocate", flush=True)
    lat = xy.Lattices(dict(L=L, beta=beta, seed=seed, rep=rep))
    assert lat.bytes < 100 * 2 ** 30
    # the merge schedule the autotuner picks for this lattice's PCC workload
    # (hash deduplication, 4 tile edges per merge wave); the default one is
    # covered on the 64-bit kernels by the wide-index parity tests
    lat.set_merge(2, 4)
    lat.sweep(1)  # sweep 0 from the hot start
    torch.cuda.synchronize()
    dev = lat.arena.device

    # seeded sample: random sites plus tile-edge and wrap-around sites
    rng = np.random.default_rng(0x65536)
    xs = np.concatenate([rng.integers(0, L, 6000), np.full(500, L - 1), rng.integers(0, L // 64, 500) * 64 + 63,
                         rng.integers(0, L, 1000)])
    ys = np.concatenate([rng.integers(0, L, 6000), rng.integers(0, L, 500), rng.integers(0, L, 500),
                         np.full(500, L - 1), rng.integers(0, L // 32, 500) * 32 + 31])
    site = (ys.astype(np.int64) * L + xs).astype(np.int64)
    right = ys.astype(np.int64) * L + (xs + 1) % L
    down = ((ys + 1) % L).astype(np.int64) * L + xs
    di = torch.from_numpy(site).to(dev)
    dr = torch.from_numpy(right).to(dev)
    dd = torch.from_numpy(down).to(dev)

    v = lat.views()
    assert v["label_bits"] == 64 and v["sweep"] == 1
    c, s = v["cos"], v["sin"]
    pre_ci, pre_si = c.index_select(0, di).double().cpu().numpy(), s.index_select(0, di).double().cpu().numpy()
    pre_cr, pre_sr = c.index_select(0, dr).double().cpu().numpy(), s.index_select(0, dr).double().cpu().numpy()
    pre_cd, pre_sd = c.index_select(0, dd).double().cpu().numpy(), s.index_select(0, dd).double().cpu().numpy()

    print("L=65536 sweep 1", flush=True)
    t = 1
    r = oracle.direction(seed, rep, t)
    assert np.array_equal(lat.sweep_count()[1], r)
    tr = lat.sweep(1, trace=True)
    torch.cuda.synchronize()
    v = lat.views()
    assert v["sweep"] == 2
    bxw, byw = v["bx"], v["by"]
    lab = lat.labels_device(bits=64)  # canonical: the smallest site of each cluster

    # 1. sampled link decisions against the oracle, from the pre-sweep spins
    def gather_bits(words, ix):
        w = words.index_select(0, ix // 32)
        return ((w >> (ix % 32).int()) & 1).cpu().numpy().astype(np.uint8)

    gx, gy = gather_bits(bxw, di), gather_bits(byw, di)
    n = site.size
    ox, tx = oracle.links(L, site, np.zeros(n, np.uint8), pre_ci, pre_si, pre_cr, pre_sr, beta, r, seed, rep, t)
    oy, ty = oracle.links(L, site, np.ones(n, np.uint8), pre_ci, pre_si, pre_cd, pre_sd, beta, r, seed, rep, t)
    # a near tie (|u - p| < 1e-9) could legitimately differ; none is expected
    # among 16000 links, and then every decision must agree
    assert tx + ty == 0
    assert np.array_equal(gx, ox), np.flatnonzero(gx != ox)[:10]
    assert np.array_equal(gy, oy), np.flatnonzero(gy != oy)[:10]
    assert gx.sum() > 0 and gy.sum() > 0

    # 2. sampled reflections: the oracle flips the sampled sites given their roots
    roots_i = lab.index_select(0, di)
    side = int(np.sqrt(n))
    m = side * side
    ri = roots_i.cpu().numpy()
    exp_c, exp_s = oracle.flip(side, ri[:m], pre_ci[:m], pre_si[:m], r, seed, rep, t)
    post_c = c.index_select(0, di).double().cpu().numpy()
    post_s = s.index_select(0, di).double().cpu().numpy()
    assert np.array_equal(post_c[:m], exp_c) and np.array_equal(post_s[:m], exp_s)
    flipped = post_c[:m] != pre_ci[:m]
    assert 0.2 < flipped.mean() < 0.8

    # 3. label forest properties and link consistency, whole lattice, by row blocks
    print("L=65536 invariants", flush=True)
    rows = 1024
    ar_cache = None
    n_active = 0
    for y0 in range(0, L, rows):
        lo, cnt = y0 * L, rows * L
        if ar_cache is None:
            ar_cache = torch.arange(cnt, device=dev, dtype=torch.int64)
        idx = ar_cache + lo
        root = lab[lo:lo + cnt]
        assert bool((root <= idx).all()), y0
        assert bool((lab.index_select(0, root) == root).all()), y0
        rr = root.view(rows, L)
        ax = _bits(bxw, lo, cnt).view(rows, L)
        assert bool((rr[ax] == rr.roll(-1, dims=1)[ax]).all()), ("x links", y0)
        y1 = (y0 + rows) % L
        down_roots = torch.cat([rr[1:], lab[y1 * L:(y1 + 1) * L].view(1, L)], dim=0)
        ay = _bits(byw, lo, cnt).view(rows, L)
        assert bool((rr[ay] == down_roots[ay]).all()), ("y links", y0)
        n_active += int(ax.sum()) + int(ay.sum())
        del root, rr, ax, ay, down_roots, idx
    assert 0 < n_active < 2 * N

    # 3b. no over-merging: host BFS of sampled clusters of at most 1e5 sites
    print("L=65536 over-merge check", flush=True)
    rng2 = np.random.default_rng(0x0E6E)
    cand = np.concatenate([rng2.integers(0, N, 120),
                           (L - 1 - rng2.integers(0, 256, 80)) * L + rng2.integers(0, L, 80)])
    checked = high = 0
    for cs in cand:
        cs = int(cs)
        lbl = int(lab[cs])
        cnt = int((lab == lbl).sum())
        if cnt > 100000:
            continue
        members = host_cluster(bxw, byw, L, cs)
        if members is None:
            continue
        assert members.size == cnt, (cs, lbl, members.size, cnt)
        assert int(members.min()) == lbl, (cs, lbl, int(members.min()))
        got = lab.index_select(0, torch.from_numpy(members).to(dev))
        assert bool((got == lbl).all()), (cs, lbl)
        checked += 1
        high += cs >= (L - 256) * L
        if checked >= 60 and high >= 20:
            break
    print("over-merge check: %d clusters (%d in the bottom rows)" % (checked, high), flush=True)
    assert checked >= 50 and high >= 10

    # 4. unit spins and observables from an FP64 recomputation of the sums
    print("L=65536 observables", flush=True)
    sums = np.zeros(6)
    colc = torch.zeros(L, dtype=torch.float64, device=dev)
    cols = torch.zeros(L, dtype=torch.float64, device=dev)
    norm_dev = 0.0
    for y0 in range(0, L, rows):
        lo, cnt = y0 * L, rows * L
        cb = c[lo:lo + cnt].double().view(rows, L)
        sb = s[lo:lo + cnt].double().view(rows, L)
        y1 = (y0 + rows) % L
        cd = torch.cat([cb[1:], c[y1 * L:(y1 + 1) * L].double().view(1, L)], 0)
        sd = torch.cat([sb[1:], s[y1 * L:(y1 + 1) * L].double().view(1, L)], 0)
        cr, sr = cb.roll(-1, dims=1), sb.roll(-1, dims=1)
        sums += np.array([float((cb * cr + sb * sr).sum()), float((sb * cr - cb * sr).sum()),
                          float((cb * cd + sb * sd).sum()), float((sb * cd - cb * sd).sum()),
                          float(cb.sum()), float(sb.sum())])
        norm_dev = max(norm_dev, float((cb * cb + sb * sb - 1.0).abs().max()))
        colc += cb.sum(dim=0)
        cols += sb.sum(dim=0)
    assert norm_dev < 1e-6
    scx, ssx, scy, ssy, sc, ss = sums
    ref = {"E": -(scx + scy) / N, "m2": (sc * sc + ss * ss) / (N * float(N)), "ex": scx / N, "sx": ssx / N,
           "ey": scy / N, "sy": ssy / N}
    ref["ups_x"] = ref["ex"] - beta * N * ref["sx"] ** 2
    kx = 2.0 * np.pi * np.arange(L) / L
    cc, cs = colc.cpu().numpy(), cols.cpu().numpy()
    ref["mk2"] = (np.dot(cc, np.cos(kx)) ** 2 + np.dot(cc, np.sin(kx)) ** 2 + np.dot(cs, np.cos(kx)) ** 2
                  + np.dot(cs, np.sin(kx)) ** 2) / float(N) ** 2
    g = tr[0, 0]
    for name in NAMES:
        assert abs(float(g[name]) - ref[name]) <= OBS_TOL, (name, float(g[name]), ref[name])
    assert -2.0 < float(g["E"]) < 0.0
    del v, lab, bxw, byw, c, s
    lat.close()
    del lat
    torch.cuda.empty_cache()
