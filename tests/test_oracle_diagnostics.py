"""Pins of the oracle's run diagnostics (Sec. 3.1.5 distributions over density,
Sec. 3.1.4 Thomson optical depth):

  * the log-uniform edges start at 10^lo, end at 10^hi and grow by the
    constant factor 10^w;
  * bin decisions agree with a brute-force scan of the edges on random
    values, on values exactly at edges (upper bin), and on out-of-range
    values (clamped into the end bins, zero included);
  * counts agree with numpy's histogram2d of log10 values away from edges
    and sum to the number of cells; per-bin sums agree with brute force;
  * tau of fully ionised uniform gas over time t is c sigma_T nH t, and
    neutral gas adds nothing."""

import math

import numpy as np
import pytest

from oracle import diagnostics as D

C = 2.99792458e10


def test_edges_geometry():
    e = D.log_edges(-6.0, 1.0, 56)
    assert len(e) == 57
    assert e[0] == pytest.approx(1e-6, rel=1e-15)
    assert e[-1] == pytest.approx(10.0, rel=1e-14)
    r = e[1:] / e[:-1]
    assert np.allclose(r, 10 ** (7.0 / 56), rtol=1e-13)


def _brute(v, e):
    nb = len(e) - 1
    k = 0
    for j in range(nb):
        if e[j] <= v:
            k = j
    return k


def test_bin_index_brute_force():
    rng = np.random.default_rng(3)
    e = D.log_edges(-5.0, 0.0, 20)
    v = 10 ** rng.uniform(-6, 1, 3000)
    got = D.bin_index(v, e)
    want = np.array([_brute(x, e) for x in v])
    assert np.array_equal(got, want)
    # exactly at an edge: the upper bin; out of range and zero: end bins
    assert list(D.bin_index(e[:-1], e)) == list(range(20))
    assert D.bin_index(np.array([0.0, 1e-30, e[0] * (1 - 1e-15)]), e).tolist() == [0, 0, 0]
    assert D.bin_index(np.array([e[-1], 1e30]), e).tolist() == [19, 19]


def test_histogram_matches_numpy_away_from_edges():
    rng = np.random.default_rng(4)
    n = 20000
    nH = 10 ** rng.uniform(-5.5, -0.5, n)
    q = 10 ** rng.uniform(-7.0, 0.0, n)
    xr, yr = (-6.0, 0.0, 24), (-8.0, 0.0, 32)
    counts, sums = D.histogram2d(nH, q, xr, yr)
    assert counts.sum() == n
    ref, _, _ = np.histogram2d(np.log10(nH), np.log10(q),
                               bins=[np.linspace(*xr[:2], xr[2] + 1),
                                     np.linspace(*yr[:2], yr[2] + 1)])
    # away from bin edges the two bin decisions coincide
    assert np.abs(counts - ref).sum() <= 2
    bx = D.bin_index(nH, D.log_edges(*xr))
    want = np.array([q[bx == k].sum() for k in range(xr[2])])
    assert np.allclose(sums, want, rtol=1e-13, atol=0)


def test_photoionisation_rate():
    assert D.photoionisation_rate(np.array([2.0]), C, 2.93e-18)[0] == (C * 2.93e-18) * 2.0


def test_thomson_closed_forms():
    nH, t = 2e-4, 3.15e16                         # ~1 Gyr of fully ionised gas
    n = (8, 8, 8)
    tau = D.thomson_increment(np.full(n, nH), np.full(n, 0.0), t, C)
    assert tau == pytest.approx(C * D.SIGMA_T * nH * t, rel=1e-14)
    assert D.thomson_increment(np.full(n, nH), np.full(n, 1.0), t, C) == 0.0
    # half the cells ionised: half the depth
    x = np.ones(n)
    x[:4] = 0.0
    assert D.thomson_increment(np.full(n, nH), x, t, C) == pytest.approx(0.5 * tau, rel=1e-14)
    assert D.SIGMA_T == pytest.approx(6.652e-25, rel=1e-4)
    assert math.isfinite(tau)
