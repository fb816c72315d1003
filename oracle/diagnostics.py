"""FP64 reference of the run diagnostics (TEST INFRASTRUCTURE ONLY: loaded by
the tests and nothing else; shares no code with the HIP path).

Sec. 3.1.5 studies the distribution of cells over density and neutral
fraction, (1 - x)(nH), and over density and ionising intensity, J21(nH),
together with the mean of each quantity per density bin.  Sec. 3.1.4 measures
the Thomson optical depth tau = c sigma_T int n_e dt.

Binning (the definition both sides implement): nb bins between 10^lo and
10^hi, uniform in log10, with edges e_k = 10^(lo + k w), w = (hi - lo) / nb,
k = 0..nb, each evaluated in FP64 as pow(10, lo + k * w).  A value v falls
in the largest k in [0, nb) with e_k <= v; values below e_0 (zero included)
fall in bin 0 and values at or above e_nb in bin nb - 1.
"""

from __future__ import annotations

import numpy as np

SIGMA_T = 6.6524587321e-25   # Thomson cross-section [cm^2] (CODATA 2018)


def log_edges(lo: float, hi: float, nb: int) -> np.ndarray:
    """The nb + 1 edges, each from the host libm's pow (as Python's float
    power)."""
    w = (hi - lo) / nb
    return np.array([10.0 ** (lo + k * w) for k in range(nb + 1)], dtype=np.float64)


def bin_index(v: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Largest k with edges[k] <= v, clamped to [0, nb - 1]."""
    nb = len(edges) - 1
    k = np.searchsorted(edges, np.asarray(v, dtype=np.float64), side="right") - 1
    return np.clip(k, 0, nb - 1)


def histogram2d(nH, q, xrange, yrange):
    """Counts (nbx, nby) of cells over (nH, q) and the per-nH-bin sum of q.

    xrange = (lo, hi, nb) for log10 nH, yrange = (lo, hi, nb) for log10 q."""
    ex = log_edges(*xrange)
    ey = log_edges(*yrange)
    nH = np.asarray(nH, dtype=np.float64).ravel()
    q = np.asarray(q, dtype=np.float64).ravel()
    bx = bin_index(nH, ex)
    by = bin_index(q, ey)
    counts = np.zeros((xrange[2], yrange[2]), dtype=np.int64)
    np.add.at(counts, (bx, by), 1)
    sums = np.zeros(xrange[2], dtype=np.float64)
    np.add.at(sums, bx, q)
    return counts, sums


def photoionisation_rate(N, c, sigma_n):
    """Gamma = c sigma_n N [1/s] per cell (Sec. 2.2 gray constants), the
    product taken as (c * sigma_n) * N in FP64."""
    return (c * sigma_n) * np.asarray(N, dtype=np.float64)


def thomson_increment(nH, xHI, dt, c):
    """c sigma_T <n_e> dt with n_e = nH (1 - xHI), the volume mean over
    cells (Sec. 3.1.4, one step of the time integral)."""
    nH = np.asarray(nH, dtype=np.float64)
    ne = nH * (1.0 - np.asarray(xHI, dtype=np.float64))
    return c * SIGMA_T * float(ne.mean()) * dt
