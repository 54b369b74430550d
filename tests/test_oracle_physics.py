"""Physics pins of the Swendsen-Wang oracle.

Nothing here re-types the oracle's formulas: each test checks a property fixed
independently of it -- limits of the bond probability (beta = 0, beta -> inf),
the geometry of a reflection, exact L = 2 averages from a character expansion and
from quadrature, an unrelated Metropolis chain at L = 8, and the fixed point of
the PCC controller measured with that Metropolis chain.
"""
import numpy as np
import pytest

import exact_l2
import oracle
import xystats
import xyworkloads as wl

OBS = {name: k for k, name in enumerate(oracle.OBS_NAMES)}


def test_beta_zero_no_bonds_identity_labels():
    L = 8
    lat = oracle.Lattice(L=L, beta=0.0, seed=3)
    for _ in range(5):
        _, ties, bx, by, lab = lat.sweep_detail()
        assert bx.sum() == 0 and by.sum() == 0
        assert np.array_equal(lab, np.arange(L * L))


def test_beta_zero_averages():
    # Independent uniform spins: <E> = 0 and <m^2> = 1/N exactly.
    L = 8
    lat = oracle.Lattice(L=L, beta=0.0, seed=4)
    tr, _ = lat.run(40000)
    for name, want in (("E", 0.0), ("m2", 1.0 / (L * L)), ("ex", 0.0), ("sx", 0.0)):
        m, e = xystats.mean_err(tr[:, OBS[name]])
        assert abs(m - want) < 3 * e, (name, m, e, want)


def test_beta_infinite_clusters_are_same_sign_domains():
    # p -> 1 when (s_i.r)(s_j.r) > 0 and p = 0 otherwise: the clusters are the
    # connected domains of equal sign of s.r.
    L = 16
    c, s = wl.random_spins(L, seed=99)
    c = c.astype(np.float64)
    s = s.astype(np.float64)
    r = oracle.direction(7, 0, 0)
    bx, by, _ = oracle.bonds(L, c, s, 1e9, r, 7, 0, 0)
    sign = (c * r[0] + s * r[1]) > 0
    idx = np.arange(L * L)
    right = (idx // L) * L + (idx % L + 1) % L
    down = ((idx // L + 1) % L) * L + idx % L
    assert np.array_equal(bx.astype(bool), sign == sign[right])
    assert np.array_equal(by.astype(bool), sign == sign[down])
    # and beta = 0 gives no bonds at all
    bx0, by0, _ = oracle.bonds(L, c, s, 0.0, r, 7, 0, 0)
    assert bx0.sum() == 0 and by0.sum() == 0


def test_sampled_links_match_whole_lattice_decisions():
    # the one-link form (used on samples of lattices too large to copy) takes
    # every decision as the whole-lattice pass does, at every site and both
    # directions, including the wrap-around links of the last row and column
    L, beta, seed, rep, t = 16, 1.12, 0x5A11, 3, 7
    c, s = wl.random_spins(L, seed=17)
    c = c.astype(np.float64)
    s = s.astype(np.float64)
    r = oracle.direction(seed, rep, t)
    bx, by, ties = oracle.bonds(L, c, s, beta, r, seed, rep, t)
    idx = np.arange(L * L)
    right = (idx // L) * L + (idx % L + 1) % L
    down = ((idx // L + 1) % L) * L + idx % L
    site = np.concatenate([idx, idx])
    dirs = np.concatenate([np.zeros(L * L), np.ones(L * L)]).astype(np.uint8)
    nb = np.concatenate([right, down])
    act, ties1 = oracle.links(L, site, dirs, c[site], s[site], c[nb], s[nb], beta, r, seed, rep, t)
    assert np.array_equal(act[:L * L], bx) and np.array_equal(act[L * L:], by)
    assert ties1 == ties
    # and in the beta -> infinity limit a sampled link is active iff the end
    # spins project on r with the same sign
    a = c * r[0] + s * r[1]
    act_inf, _ = oracle.links(L, site, dirs, c[site], s[site], c[nb], s[nb], 1e9, r, seed, rep, t)
    assert np.array_equal(act_inf.astype(bool), (a[site] > 0) == (a[nb] > 0))


def test_bond_fraction_grows_with_beta():
    L = 32
    c, s = wl.random_spins(L, seed=5)
    r = oracle.direction(1, 0, 0)
    fr = [sum(x.sum() for x in oracle.bonds(L, c, s, b, r, 1, 0, 0)[:2]) for b in (0.1, 0.5, 1.0, 4.0)]
    assert fr == sorted(fr) and fr[0] < fr[-1]


def test_reflection_geometry_and_cluster_coherence():
    L = 16
    lat = oracle.Lattice(L=L, beta=1.12, seed=21)
    lat.run(3)
    c0, s0 = lat.c.copy(), lat.s.copy()
    t = lat.t
    r = oracle.direction(lat.seed, lat.rep, t)
    _, _, bx, by, lab = lat.sweep_detail()
    c1, s1 = lat.c, lat.s
    par0 = c0 * r[0] + s0 * r[1]
    par1 = c1 * r[0] + s1 * r[1]
    perp0 = -c0 * r[1] + s0 * r[0]
    perp1 = -c1 * r[1] + s1 * r[0]
    flipped = np.array([oracle.coin(lat.seed, lat.rep, t, int(x)) for x in lab], dtype=bool)
    # flipped sites: component along r reversed, perpendicular kept
    assert np.allclose(par1[flipped], -par0[flipped], atol=3e-7)
    assert np.allclose(perp1[flipped], perp0[flipped], atol=3e-7)
    # unflipped sites untouched
    assert np.array_equal(c1[~flipped], c0[~flipped]) and np.array_equal(s1[~flipped], s0[~flipped])
    # unit length kept
    assert np.max(np.abs(np.hypot(c1, s1) - 1.0)) < 1e-6
    # a cluster flips as a whole: both ends of an active link share the decision
    idx = np.arange(L * L)
    right = (idx // L) * L + (idx % L + 1) % L
    down = ((idx // L + 1) % L) * L + idx % L
    assert np.all(flipped[bx.astype(bool)] == flipped[right[bx.astype(bool)]])
    assert np.all(flipped[by.astype(bool)] == flipped[down[by.astype(bool)]])
    # active links join spins on the same side of the mirror line
    assert np.all(par0[bx.astype(bool)] * par0[right[bx.astype(bool)]] > 0)


def test_measure_matches_angle_formulas():
    # The oracle's observables from (cos, sin) against cos/sin of angle
    # differences evaluated here from the angles.
    L = 8
    rng = np.random.default_rng(3)
    th = rng.uniform(0, 2 * np.pi, L * L)
    beta = 0.9
    obs = oracle.measure(L, np.cos(th), np.sin(th), beta)
    T = th.reshape(L, L)
    dx = T - np.roll(T, -1, axis=1)
    dy = T - np.roll(T, -1, axis=0)
    N = L * L
    want = [-(np.cos(dx).sum() + np.cos(dy).sum()) / N,
            (np.cos(T).sum() ** 2 + np.sin(T).sum() ** 2) / N ** 2,
            np.cos(dx).sum() / N, np.sin(dx).sum() / N, np.cos(dy).sum() / N, np.sin(dy).sum() / N]
    want.append(want[2] - beta * N * want[3] ** 2)
    # chi(k)/N at k = 2 pi / L along x, from a library FFT of each component
    fc = np.fft.fft(np.cos(T), axis=1)[:, 1].sum()
    fs = np.fft.fft(np.sin(T), axis=1)[:, 1].sum()
    want.append((abs(fc) ** 2 + abs(fs) ** 2) / N ** 2)
    assert np.allclose(obs, want, atol=1e-13)


def test_fourier_magnetisation_closed_forms():
    # a spin wave of wave vector (2 pi / L, 0) has |sum s e^{ikx}|^2 = N^2 / 2
    # and no magnetisation; a uniform state the reverse; a wave along y has
    # no weight at k along x
    L = 16
    N = L * L
    x = np.tile(np.arange(L), L)
    y = np.repeat(np.arange(L), L)
    for th, m2, mk2 in ((2 * np.pi * x / L, 0.0, 0.5), (np.full(N, 0.7), 1.0, 0.0),
                        (2 * np.pi * y / L, 0.0, 0.0), (-2 * np.pi * x / L, 0.0, 0.5)):
        obs = oracle.measure(L, np.cos(th), np.sin(th), 1.0)
        assert abs(obs[OBS["m2"]] - m2) < 1e-13 and abs(obs[OBS["mk2"]] - mk2) < 1e-13


@pytest.mark.parametrize("beta", [0.5, 1.12])
def test_l2_exact_averages(beta):
    ex = exact_l2.character_expansion(beta)
    q = exact_l2.quadrature(beta)
    for k in ex:
        assert abs(ex[k] - q[k]) < 1e-12
    lat = oracle.Lattice(L=2, beta=beta, seed=0xC0FFEE + int(beta * 100))
    lat.run(1000)
    tr, _ = lat.run(400000)
    assert np.all(tr[:, OBS["sx"]] == 0.0)
    for name in ("E", "m2", "ex", "ups_x"):
        m, e = xystats.mean_err(tr[:, OBS[name]])
        assert abs(m - ex[name]) < 3 * e, (name, m, e, ex[name])


@pytest.mark.parametrize("beta", [0.8, 1.12])
def test_l8_agrees_with_metropolis(beta):
    L = 8
    lat = oracle.Lattice(L=L, beta=beta, seed=0x5EED + int(beta * 100))
    lat.run(1000)
    tr_sw, _ = lat.run(100000)
    tr_m, acc, _ = oracle.metropolis(L, beta, 200000, ntherm=5000, seed=77 + int(beta * 100),
                                     delta=2.0)
    assert 0.2 < acc < 0.8
    cols_m = {"E": 0, "m2": 1, "ex": 2, "ups_x": 4}
    for name, km in cols_m.items():
        a, ea = xystats.mean_err(tr_sw[:, OBS[name]])
        b, eb = xystats.mean_err(tr_m[:, km])
        assert xystats.agree(a, ea, b, eb, 3.0), (name, a, ea, b, eb)


def test_pcc_fixed_point_matches_metropolis_helicity():
    # The PCC chain settles where beta*Upsilon(beta) = 0.636508.  Run the oracle's
    # controller at L = 8, then measure beta*Upsilon with the Metropolis chain at
    # the mean beta it found.
    L = 8
    lat = oracle.Lattice(L=L, beta=1.0, seed=0xACC)
    lat.pcc(200, 100, 0.01)                       # settle
    betas, bu = lat.pcc(1500, 100, 0.002)         # measure
    b_star, b_err = xystats.mean_err(betas, nbins=30)
    assert 0.9 < b_star < 1.3
    tr_m, _, _ = oracle.metropolis(L, b_star, 300000, ntherm=5000, seed=4242)
    u, ue = xystats.mean_err(b_star * tr_m[:, 4])
    assert abs(u - oracle.PCC_TARGET) < 3 * ue + 0.01, (b_star, u, ue)


def test_pcc_direction_of_steps():
    # Far below the KT point (beta small) beta*Upsilon is small, so beta must rise;
    # far above it beta*Upsilon is large, so beta must fall.
    lo = oracle.Lattice(L=8, beta=0.3, seed=1)
    b_lo, _ = lo.pcc(20, 50, 0.01)
    assert np.all(np.diff(np.concatenate([[0.3], b_lo])) > 0)
    hi = oracle.Lattice(L=8, beta=3.0, seed=2)
    b_hi, _ = hi.pcc(20, 50, 0.01)
    assert np.all(np.diff(np.concatenate([[3.0], b_hi])) < 0)


def test_pcc_halving_schedule():
    lat = oracle.Lattice(L=4, beta=0.3, seed=9)
    b, _ = lat.pcc(8, 5, 0.004, dbeta_min=0.0005, halve_every=2)
    steps = np.abs(np.diff(np.concatenate([[0.3], b])))
    assert np.allclose(steps, [0.004, 0.004, 0.002, 0.002, 0.001, 0.001, 0.0005, 0.0005])
