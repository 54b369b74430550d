"""Finite-size-scaling fits (paper_1210_6116_amd.fss) pinned to the paper.

The paper's Table 1 rows (tests/golden/table1.txt) fitted with Eq. (beta_KT)
give its printed line 1.11996 - 0.826 l^-2 at b = 3.6 (the caption of the
beta_KT(L) figure, minimum sizes 128 and 256) and the estimate beta_KT =
1.11996; the log-correction fit of <m^2>_L with a = 16 gives -2r = 0.128(8).
Closed-form data generated from the models pin the algebra itself.
"""
import math
import os

import numpy as np
import pytest

from paper_1210_6116_amd import fss

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def _table():
    d = np.loadtxt(GOLDEN)
    return d[:, 0], d[:, 1], d[:, 2], d[:, 3], d[:, 4]


def test_weighted_line_recovers_exact_line_and_errors():
    x = np.array([0.0, 1.0, 2.0, 3.0])
    f = fss.weighted_line(x, 2.0 - 0.5 * x, np.ones(4))
    assert f.intercept == pytest.approx(2.0, abs=1e-14) and f.slope == pytest.approx(-0.5, abs=1e-14)
    assert f.chi2 == pytest.approx(0.0, abs=1e-24) and f.dof == 2
    # unit weights: var(slope) = 1 / sum (x - mean)^2 = 1/5
    assert f.slope_err == pytest.approx(math.sqrt(1 / 5.0))
    # a point with a much larger error barely moves the fit
    y = 2.0 - 0.5 * x
    y[3] += 10.0
    g = fss.weighted_line(x, y, np.array([1.0, 1.0, 1.0, 1e6]))
    assert g.slope == pytest.approx(-0.5, abs=1e-9)


def test_beta_kt_fit_on_synthetic_kt_form():
    L = 2.0 ** np.arange(6, 17)
    bkt, c2, b = 1.12, 0.74, 3.6
    beta = bkt - c2 * bkt / np.log(b * L) ** 2
    f = fss.fit_beta_kt(L, beta, np.full(L.size, 1e-4), b)
    assert f.beta_kt == pytest.approx(bkt, abs=1e-12)
    assert f.c2 == pytest.approx(c2, abs=1e-10)
    assert f.chi2 == pytest.approx(0.0, abs=1e-12)
    # the scan finds the b the data were made with
    assert fss.best_b(L, beta, np.full(L.size, 1e-4)).b == pytest.approx(b, abs=0.005)


def test_beta_kt_fit_reproduces_the_paper():
    L, beta, err, _, _ = _table()
    for lmin in (128, 256):
        sel = L >= lmin
        f = fss.fit_beta_kt(L[sel], beta[sel], err[sel], 3.6)
        # the printed line: 1.11996 - 0.826 l^-2, beta_KT = 1.11996(6)
        assert abs(f.beta_kt - 1.11996) < 2 * f.beta_kt_err, (lmin, f)
        assert abs(f.slope + 0.826) < 2 * f.slope_err, (lmin, f)
        assert f.chi2 / f.dof < 1.0
        g = fss.best_b(L[sel], beta[sel], err[sel])
        assert 3.0 < g.b < 4.5, g


def test_log_correction_on_synthetic_data():
    L = 2.0 ** np.arange(6, 17)
    a, m2r = 16.0, 0.125
    m2 = 1.3 * np.log(a * L) ** m2r * L ** -0.25
    f = fss.fit_log_correction(L, m2, 1e-4 * m2, a)
    assert f.minus_2r == pytest.approx(m2r, abs=1e-12)
    assert f.const == pytest.approx(math.log(1.3), abs=1e-12)


def test_log_correction_reproduces_the_paper():
    L, _, _, m2, err = _table()
    f = fss.fit_log_correction(L, m2, err, 16.0)
    assert abs(f.minus_2r - 0.128) < 0.008, f  # -2r = 0.128(8)
    # a = 1: the slope is smaller on small lattices than on large ones, and
    # approaches 1/8 from below
    small = (L >= 64) & (L <= 2048)
    large = (L >= 2048) & (L <= 65536)
    s = fss.fit_log_correction(L[small], m2[small], err[small], 1.0).minus_2r
    g = fss.fit_log_correction(L[large], m2[large], err[large], 1.0).minus_2r
    assert 0.05 < s < g < 0.125 + 0.01, (s, g)


def test_main_prints_both_fits(capsys):
    assert fss.main([GOLDEN, "128"]) == 0
    out = capsys.readouterr().out
    assert "beta_KT = 1.11" in out and "-2r" in out
