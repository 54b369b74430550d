"""Exact thermal averages of the periodic L = 2 XY lattice (a test pin).

With periodic boundaries the L = 2 lattice has four sites; each site's right and
down links wrap onto the same neighbour, so every neighbour pair is coupled
twice and the lattice is a four-site ring with coupling K = 2 beta (Eq. (Hc)
summed literally over the 2N links).  Two independent evaluations are given:

* ``character_expansion``: exp(K cos t) = sum_m I_m(K) e^{imt} turns the ring's
  partition function into Z = sum_m I_m(K)^4, from which the nearest- and
  next-nearest-neighbour correlations follow as
  c1 = sum_m I_m^3 I_{m+1} / Z and c2 = sum_m I_m^2 I_{m+1}^2 / Z;
* ``quadrature``: the three free angles (the fourth fixed by global rotation
  symmetry) integrated on a periodic trapezoid grid.

Observables (per site, as in the oracle): E = -2 c1, m2 = (1 + 2 c1 + c2) / 4,
ex = c1, sx = 0 identically (the two x-links of each pair cancel), hence
ups_x = ex.
"""
import numpy as np
from scipy.special import iv


def character_expansion(beta: float, mmax: int = 60):
    K = 2.0 * beta
    m = np.arange(-mmax, mmax + 1)
    Im = iv(m, K)
    Im1 = iv(m + 1, K)
    Z = np.sum(Im ** 4)
    c1 = np.sum(Im ** 3 * Im1) / Z
    c2 = np.sum(Im ** 2 * Im1 ** 2) / Z
    return dict(E=-2.0 * c1, m2=(1.0 + 2.0 * c1 + c2) / 4.0, ex=c1, ups_x=c1)


def quadrature(beta: float, n: int = 64):
    K = 2.0 * beta
    t = 2.0 * np.pi * np.arange(n) / n
    t1, t2, t3 = np.meshgrid(t, t, t, indexing="ij")
    t0 = np.zeros_like(t1)
    # sites 0=(0,0) 1=(1,0) 2=(0,1) 3=(1,1); ring 0-1-3-2-0, each pair linked twice
    ring = np.cos(t0 - t1) + np.cos(t1 - t3) + np.cos(t3 - t2) + np.cos(t2 - t0)
    w = np.exp(K * ring - 4.0 * K)
    Z = w.sum()
    E = -(2.0 * ring) / 4.0
    ex = (2.0 * np.cos(t0 - t1) + 2.0 * np.cos(t2 - t3)) / 4.0
    mc = (np.cos(t0) + np.cos(t1) + np.cos(t2) + np.cos(t3)) / 4.0
    ms = (np.sin(t0) + np.sin(t1) + np.sin(t2) + np.sin(t3)) / 4.0
    m2 = mc ** 2 + ms ** 2
    avg = lambda a: float((w * a).sum() / Z)
    return dict(E=avg(E), m2=avg(m2), ex=avg(ex), ups_x=avg(ex))
