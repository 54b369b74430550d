"""Pins of the oracle's counter-based generator (Philox4x32-10, SC'11)."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(v, 16) for v in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_philox4x32_known_answers(ctr, key, want):
    assert list(oracle.philox4x32_10(ctr, key)) == want


def test_philox4x64_matches_numpy():
    # numpy's Philox is an independent implementation of the 4x64-10 member of
    # the family; it pre-increments its counter before the first block.
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = [int(v) for v in rng.integers(0, 2 ** 63, size=2)]
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, size=4)]
        bg = np.random.Philox(key=key, counter=ctr)
        raw = [int(v) for v in bg.random_raw(4)]
        ctr1 = list(ctr)
        ctr1[0] += 1
        assert [int(v) for v in oracle.philox4x64_10(ctr1, key)] == raw


def test_philox4x32_uniform_bits():
    # Bit frequencies and a chi-square of the top byte over 4096 counters.
    words = np.array([oracle.philox4x32_10([i, 3, 5, 1], [0x12345678, 0x9ABCDEF0])
                      for i in range(4096)], dtype=np.uint64).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(words.size))
    counts = np.bincount((words >> 24).astype(np.int64), minlength=256)
    exp = words.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 255 + 5 * np.sqrt(2 * 255)


def test_direction_uniform_and_unit():
    r = np.array([oracle.direction(0xABC, 1, t) for t in range(8000)])
    assert np.max(np.abs(np.hypot(r[:, 0], r[:, 1]) - 1.0)) < 4e-16
    ang = np.arctan2(r[:, 1], r[:, 0])
    counts, _ = np.histogram(ang, bins=16, range=(-np.pi, np.pi))
    exp = len(ang) / 16
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 15 + 5 * np.sqrt(30)
    # streams of different replicas / sweeps are different
    assert not np.allclose(oracle.direction(0xABC, 1, 5), oracle.direction(0xABC, 2, 5))


def test_hot_start_uniform_angles():
    L = 64
    c, s = oracle.hot_start(L, 0x12106116, 0, storage32=True)
    assert np.all(c.astype(np.float32).astype(np.float64) == c)
    assert np.max(np.abs(np.hypot(c, s) - 1.0)) < 2e-7
    ang = np.arctan2(s, c)
    counts, _ = np.histogram(ang, bins=32, range=(-np.pi, np.pi))
    exp = len(ang) / 32
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 31 + 5 * np.sqrt(62)
    # the net magnetisation of N independent unit vectors is O(1/sqrt(N))
    assert np.hypot(c.mean(), s.mean()) < 5.0 / np.sqrt(L * L)


def test_coin_fair_and_root_keyed():
    coins = np.array([oracle.coin(11, 0, 3, r) for r in range(20000)])
    assert abs(coins.mean() - 0.5) < 5 * 0.5 / np.sqrt(coins.size)
    assert oracle.coin(11, 0, 3, 777) == oracle.coin(11, 0, 3, 777)
