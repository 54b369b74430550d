"""Error bars for Markov-chain time series (binning / blocking analysis).

A series of correlated samples is cut into `nbins` consecutive blocks; once the
blocks are much longer than the integrated autocorrelation time the block means
are nearly independent, and their spread gives the error of the overall mean.
"""
import numpy as np


def mean_err(x, nbins: int = 40):
    x = np.asarray(x, dtype=np.float64)
    n = (len(x) // nbins) * nbins
    blocks = x[:n].reshape(nbins, -1).mean(axis=1)
    return float(x.mean()), float(blocks.std(ddof=1) / np.sqrt(nbins))


def tau_int(x, wmax: int = 200):
    """Integrated autocorrelation time with Madras-Sokal self-consistent window (c = 6)."""
    x = np.asarray(x, dtype=np.float64) - np.mean(x)
    var = np.dot(x, x) / len(x)
    if var == 0:
        return 0.5
    tau = 0.5
    for w in range(1, min(wmax, len(x) // 2)):
        rho = np.dot(x[:-w], x[w:]) / (len(x) - w) / var
        tau += rho
        if w >= 6 * tau:
            break
    return max(tau, 0.5)


def agree(a, ea, b, eb, nsigma: float = 3.0) -> bool:
    return abs(a - b) <= nsigma * np.sqrt(ea * ea + eb * eb)
