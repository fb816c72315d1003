"""GPU checks of the run diagnostics through the C ABI against the FP64
oracle (Sec. 3.1.5 distributions over density, Sec. 3.1.4 Thomson depth):

  * rt_histogram counts equal the oracle's exactly (integer work) for the
    neutral fraction and the photoionisation rate, on an evolved
    cosmological state, on a ragged grid, at the largest bin count and for
    a single bin; values exactly on edges and out of range land where the
    definition puts them; per-density-bin sums agree to 1e-12;
  * tau_e: closed form for a frozen uniform state (c sigma_T <n_e> t), and
    the oracle's step-by-step sum on a Stromgren run."""

import numpy as np
import pytest
import torch

import oracle
from oracle import diagnostics as D
from paper_1004_2503_amd import rt
from paper_1004_2503_amd import workloads as W

from parity_util import oracle_grid

pytestmark = pytest.mark.gpu

C = rt.C_LIGHT


def check_hist(G, st, quantity, xr, yr):
    counts, sums = G.histogram(quantity, xr, yr)
    q = st["xHI"] if quantity == rt.HQ_XHI else D.photoionisation_rate(st["N"], C, rt.SIGMA_N)
    oc, osum = D.histogram2d(st["nH"], q, xr, yr)
    assert counts.shape == oc.shape
    assert np.array_equal(counts, oc), np.argwhere(counts != oc)[:5]
    assert np.allclose(sums, osum, rtol=1e-12, atol=0.0)
    return counts


@pytest.fixture(scope="module")
def evolved64():
    n = 64
    dx = W.cosmo_dx(n)
    nH = W.lognormal_density(n).numpy()
    ijk = W.densest_cells(torch.from_numpy(nH), 64)
    G = rt.RTGrid(rt.make_params((n,) * 3, dx, prec=rt.PREC_MIXED), dict(nH=nH))
    G.inject_sources(ijk, W.luminosities(len(ijk)))
    G.step(W.courant_dt(dx), 1, 80)
    st = G.state_numpy()
    yield G, st
    G.close()


@pytest.mark.parametrize("quantity", [rt.HQ_XHI, rt.HQ_GAMMA])
@pytest.mark.parametrize("nb", [(64, 128), (1, 1), (40, 7)])
def test_histogram_counts_exact_on_evolved_state(evolved64, quantity, nb):
    G, st = evolved64
    yr = (-7.0, 0.5, nb[1]) if quantity == rt.HQ_XHI else (-16.0, -8.0, nb[1])
    counts = check_hist(G, st, quantity, (-6.0, 0.0, nb[0]), yr)
    assert counts.sum() == st["nH"].size
    if nb == (64, 128):
        assert np.count_nonzero(counts) > 50      # a spread distribution


def test_histogram_edges_range_and_ragged_grid():
    shape = (37, 29, 70)                     # 75110 cells: a ragged last block
    st = W.random_state(shape, seed=91, nH_range=(1e-3, 3e2), nmax=1e-8)
    # values exactly on edges (10^k are FP64 edges of the range below and
    # exactly representable as floats only at k >= 0), and out of range
    flat = st["nH"].reshape(-1)
    flat[:5] = [1.0, 10.0, 100.0, 1e-9, 5e3]
    st["N"].reshape(-1)[:3] = 0.0            # Gamma = 0 -> bin 0
    G = rt.RTGrid(rt.make_params(shape, 1e21), st)
    xr = (-2.0, 2.0, 4)                       # edges 0.01, 0.1, 1, 10, 100
    counts = check_hist(G, st, rt.HQ_XHI, xr, (-6.0, 0.0, 12))
    bx = D.bin_index(flat[:5], D.log_edges(*xr))
    assert bx.tolist() == [2, 3, 3, 0, 3]
    check_hist(G, st, rt.HQ_GAMMA, xr, (-14.0, -6.0, 16))
    G.close()
    assert counts.sum() == flat.size


def test_histogram_rejects_bad_ranges():
    shape = (4, 4, 64)
    G = rt.RTGrid(rt.make_params(shape, 1e21), W.random_state(shape, seed=1))
    for q, xr, yr in [(5, (-1, 0, 4), (-1, 0, 4)), (0, (0, 0, 4), (-1, 0, 4)),
                      (0, (-1, 0, 0), (-1, 0, 4)), (0, (-1, 0, 257), (-1, 0, 4)),
                      (0, (-1, 0, 128), (-1, 0, 128)), (0, (-400, 0, 4), (-1, 0, 4))]:
        rc, _, _ = rt.rt_histogram(G.ctx, q, xr, yr)
        assert rc == rt.RT_E_ARG, (q, xr, yr)
    G.close()


def test_thomson_depth_closed_form_frozen_state():
    # chemistry off: xHI never changes, so tau = c sigma_T <nH (1 - xHI)> t
    shape = (16, 16, 64)
    st = W.random_state(shape, seed=5, nH_range=(1e-4, 1e-2), xhi_range=(1e-3, 1.0))
    dx = 3e21
    dt = W.courant_dt(dx)
    G = rt.RTGrid(rt.make_params(shape, dx, chem=rt.CHEM_OFF), st)
    G.step(dt, 1, 7)
    red = G.reduce()
    G.close()
    ne = np.mean(st["nH"].astype(np.float64) * (1.0 - st["xHI"].astype(np.float64)))
    assert red["tau_e"] == pytest.approx(C * D.SIGMA_T * ne * 7 * dt, rel=1e-9)


def test_thomson_depth_matches_oracle_run():
    w = W.workload("stromgren32")
    n = w.n
    st = dict(xHI=np.ones((n,) * 3, np.float32), T=np.full((n,) * 3, 1e4, np.float32),
              nH=np.full((n,) * 3, w.nH_mean, np.float32))
    src = W.stromgren_sources(w)
    G = rt.RTGrid(rt.make_params((n,) * 3, w.dx, bc=w.bc, chem=rt.CHEM_ISOTHERMAL), st)
    G.inject_sources(*src)
    g = oracle_grid(st, (n,) * 3, w.dx, w.bc, oracle.CHEM_ISOTHERMAL, sources=src)
    tau_o = 0.0
    for _ in range(120):
        G.step(w.dt, 1)
        g.step(w.dt, 1)
        tau_o += D.thomson_increment(g.nH, g.xHI, w.dt, C)
    red = G.reduce()
    G.close()
    assert tau_o > 0
    assert red["tau_e"] == pytest.approx(tau_o, rel=5e-3)
