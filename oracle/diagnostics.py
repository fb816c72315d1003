"""FP64 reference of the run diagnostics (TEST INFRASTRUCTURE ONLY: loaded by
the tests and nothing else; shares no code with the HIP path).

Sec. 3.1.5 studies the distribution of cells over density and neutral
fraction, (1 - x)(nH), and over density and ionising intensity, J21(nH),
together with the mean of each quantity per density bin.  Sec. 3.1.4 measures
the Thomson optical depth tau = c sigma_T int n_e dt.

Sec. 3.1.5 also models the intensity against density by a plateau J0 with
an exponential self-shielding cutoff, J1 = J0 exp(-nH/n1*) and
J4 = J0 exp(-(nH/n4*)^4) (the printed exp((-nH/n4*)^4) would grow with
density; the cutoff the text describes is read), and compares the mean
neutral fraction per density bin with the photoionisation equilibrium under
each model.  With the gray constants the rate Gamma = c sigma_n N is
proportional to J, so the models are applied to Gamma.  The equilibrium is
the fixed point of the chemistry at fixed T and Gamma: case-B recombination
(times C_R) balances photoionisation (times C_I) and collisional ionisation,

    C_R alpha_B nH (1 - y)^2 = C_I Gamma y + beta nH (1 - y) y,

y the neutral fraction; y is its root in [0, 1], taken from the quadratic in
the cancellation-free form (the smaller root as the product of the roots over
the larger).

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


MODEL_UNIFORM, MODEL_EXP1, MODEL_EXP4 = 0, 1, 2


def gamma_model(model: int, gamma0: float, n_star: float, nH):
    """Gamma(nH) of the plateau (J0), J1 or J4 model (Sec. 3.1.5)."""
    nH = np.asarray(nH, dtype=np.float64)
    if model == MODEL_UNIFORM:
        return np.full(nH.shape, float(gamma0))
    if model == MODEL_EXP1:
        return gamma0 * np.exp(-nH / n_star)
    if model == MODEL_EXP4:
        return gamma0 * np.exp(-((nH / n_star) ** 4))
    raise ValueError(model)


def xhi_equilibrium(nH, T, gamma, params=None):
    """Equilibrium neutral fraction per element of (nH, T, gamma); params
    (oracle Params) supplies the clumping laws, None for no clumping."""
    from . import clumping, rates

    nH = np.atleast_1d(np.asarray(nH, dtype=np.float64))
    T = np.broadcast_to(np.asarray(T, dtype=np.float64), nH.shape)
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), nH.shape)
    out = np.empty(nH.shape)
    for i in np.ndindex(nH.shape):
        r = rates(float(T[i]))
        cr, ci = clumping(params, float(nH[i])) if params is not None else (1.0, 1.0)
        a = cr * r[0] * nH[i]                 # recombination
        b = r[1] * nH[i]                      # collisional ionisation
        g = ci * gamma[i]                     # photoionisation
        # (a + b) y^2 - (2a + g + b) y + a = 0.  Its roots multiply to
        # a / (a + b) <= 1; the larger is q / (a + b) with q = (-B + sqrt(disc)) / 2
        # (no cancellation: -B > 0), the wanted smaller one a / q.  The plain
        # (-B - sqrt(disc)) / 2A would lose all digits for y << 1.
        # The discriminant B^2 - 4 A a expands to (g + b)^2 + 4 a g, written
        # so: as a difference it cancels in nearly neutral gas (g + b << a).
        A, B = a + b, -(2.0 * a + g + b)
        disc = (g + b) ** 2 + 4.0 * a * g
        q = 0.5 * (-B + np.sqrt(disc))
        out[i] = a / q if q > 0.0 else 1.0
    return out


def gamma_plateau(nH, gamma, nH_max):
    """J0 as a rate: mean Gamma over the cells with nH < nH_max."""
    nH = np.asarray(nH, dtype=np.float64).ravel()
    g = np.asarray(gamma, dtype=np.float64).ravel()
    sel = nH < nH_max
    return float(g[sel].sum() / sel.sum())


def thomson_increment(nH, xHI, dt, c):
    """c sigma_T <n_e> dt with n_e = nH (1 - xHI), the volume mean over
    cells (Sec. 3.1.4, one step of the time integral)."""
    nH = np.asarray(nH, dtype=np.float64)
    ne = nH * (1.0 - np.asarray(xHI, dtype=np.float64))
    return c * SIGMA_T * float(ne.mean()) * dt
