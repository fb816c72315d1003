"""GPU checks of the run diagnostics through the C ABI against the FP64
oracle (Sec. 3.1.5 distributions over density, Sec. 3.1.4 Thomson depth):

  * rt_histogram counts equal the oracle's exactly (integer work) for the
    neutral fraction and the photoionisation rate, on an evolved
    cosmological state, on a ragged grid, at the largest bin count and for
    a single bin, on fields that are not 16-byte aligned; values exactly on
    edges and out of range land where the definition puts them;
    per-density-bin sums agree to 1e-12;
  * tau_e: closed form for a frozen uniform state (c sigma_T <n_e> t), and
    the oracle's step-by-step sum on a Stromgren run;
  * rt_equilibrium_xhi under the plateau, J1 and J4 models, with and
    without clumping, element by element against the oracle (the neutral
    and the ionised fraction to 2e-5: the kernel takes the FP32 rate fits of
    the step), invalid elements NaN, no radiation in cold gas exactly 1; and
    the analysis of Sec. 3.1.5 on an evolved state: plateau rate from the
    rate histogram, then the equilibrium curves at the bin centres."""

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


@pytest.mark.parametrize("offset", [0, 1, 2])
def test_histogram_on_unaligned_fields(offset):
    # fields that start 4 or 8 bytes past a 16-byte boundary take the
    # cell-by-cell path; the counts are the same
    shape = (5, 7, 41)                       # 1435 cells: not a multiple of 8
    n = int(np.prod(shape))
    st = W.random_state(shape, seed=17 + offset)
    buf = {k: torch.zeros(n + 4, dtype=torch.float32, device="cuda") for k in
           ("N0", "N1", "Fx0", "Fx1", "Fy0", "Fy1", "Fz0", "Fz1", "xHI", "T", "nH")}
    view = {k: v[offset:offset + n] for k, v in buf.items()}
    for k in ("xHI", "T", "nH"):
        view[k].copy_(torch.from_numpy(st[k].reshape(-1)))
    for k in ("N", "Fx", "Fy", "Fz"):
        view[k + "0"].copy_(torch.from_numpy(st[k].reshape(-1)))
    f = rt.rt_fields()
    for k in ("N", "Fx", "Fy", "Fz"):
        getattr(f, k)[0] = view[k + "0"].data_ptr()
        getattr(f, k)[1] = view[k + "1"].data_ptr()
    f.xHI, f.T, f.nH = view["xHI"].data_ptr(), view["T"].data_ptr(), view["nH"].data_ptr()
    assert (view["nH"].data_ptr() % 16 == 0) == (offset == 0)
    torch.cuda.synchronize()
    rc, ctx = rt.rt_init(rt.make_params(shape, 1e21), f, None)
    rt.check(rc, "rt_init")
    try:
        for quantity, yr in ((rt.HQ_XHI, (-7.0, 0.5, 32)), (rt.HQ_GAMMA, (-16.0, -8.0, 32))):
            xr = (-6.0, 0.0, 24)
            rc, counts, sums = rt.rt_histogram(ctx, quantity, xr, yr)
            rt.check(rc, "rt_histogram")
            q = st["xHI"] if quantity == rt.HQ_XHI else D.photoionisation_rate(st["N"], C,
                                                                               rt.SIGMA_N)
            oc, osum = D.histogram2d(st["nH"], q, xr, yr)
            assert np.array_equal(counts, oc)
            assert np.allclose(sums, osum, rtol=1e-12, atol=0.0)
    finally:
        rt.lib().rt_destroy(ctx)


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


LAW_B = W.CLUMP_LAWS["B"]


def _eq_gpu(params, model, g0, ns, nH, T):
    d = dict(dtype=torch.float64, device="cuda")
    out = rt.equilibrium_xhi(params, model, g0, ns, torch.tensor(nH, **d), torch.tensor(T, **d))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _compare_eq(y, want):
    assert np.all(np.abs(y - want) <= 2e-5 * want), np.max(np.abs(y - want) / want)
    ion_w, ion = 1.0 - want, 1.0 - y
    m = ion_w > 1e-9
    tol = 2e-5 + 1e-15 / ion_w[m]
    assert np.all(np.abs(ion[m] - ion_w[m]) <= tol * ion_w[m])


@pytest.mark.parametrize("model,ns", [(rt.JMODEL_UNIFORM, 0.0), (rt.JMODEL_EXP1, 0.007),
                                      (rt.JMODEL_EXP4, 0.018)])
@pytest.mark.parametrize("clump", [None, LAW_B])
def test_equilibrium_matches_oracle(model, ns, clump):
    rng = np.random.default_rng(40 + model)
    n = 3000
    nH = 10 ** rng.uniform(-6, 0, n)
    T = 10 ** rng.uniform(2, 5, n)
    g0 = 1e-12
    p = rt.make_params((1, 1, 1), 1e21, clump=clump)
    y = _eq_gpu(p, model, g0, ns, nH, T)
    op = oracle.make_params((1, 1, 1), 1e21, clump=clump) if clump is not None else None
    want = D.xhi_equilibrium(nH, T, D.gamma_model(model, g0, ns, nH), op)
    _compare_eq(y, want)
    # the regimes are present: ionised, partly neutral and (under a cutoff
    # or with clumping) shielded
    assert (want < 1e-4).any() and ((want > 0.01) & (want < 0.5)).any()
    if model != rt.JMODEL_UNIFORM or clump is not None:
        assert (want > 0.9).any()


def test_equilibrium_special_elements():
    p = rt.make_params((1, 1, 1), 1e21)
    nH = np.array([0.0, -1.0, np.inf, 1e-3, 1e-3, 1e-3, 1e-3, 1e-2])
    T = np.array([1e4, 1e4, 1e4, 0.5, np.nan, 2e9, 100.0, 1e4])
    y = _eq_gpu(p, rt.JMODEL_UNIFORM, 0.0, 0.0, nH, T)
    assert np.all(np.isnan(y[:6]))
    assert y[6] == 1.0                       # cold, dark: no ionisation at all
    a, b = oracle.rates(1e4)[:2]
    assert y[7] == pytest.approx(a / (a + b), rel=2e-5)   # coronal equilibrium


def test_equilibrium_curves_of_an_evolved_state(evolved64):
    G, st = evolved64
    xr, yr = (-6.0, 0.0, 48), (-18.0, -8.0, 64)
    counts, sums = G.histogram(rt.HQ_GAMMA, xr, yr)
    edges = D.log_edges(*xr)
    cut = edges[30]                                    # 10^-2.25 cm^-3
    g0, ncut = G.gamma_plateau(cut)
    gam = D.photoionisation_rate(st["N"], C, rt.SIGMA_N)
    want0 = D.gamma_plateau(st["nH"], gam, cut)
    assert g0 == pytest.approx(want0, rel=1e-12)
    assert ncut == int((np.asarray(st["nH"], np.float64) < cut).sum())
    # the same state gives the same plateau bit for bit
    assert G.gamma_plateau(cut)[0] == g0
    assert g0 > 0.0
    centres = np.sqrt(edges[:-1] * edges[1:])
    T = np.full_like(centres, 1e4)
    p = rt.make_params((1, 1, 1), 1e21)
    for model, ns in ((rt.JMODEL_UNIFORM, 0.0), (rt.JMODEL_EXP1, 0.007),
                      (rt.JMODEL_EXP4, 0.018)):
        y = _eq_gpu(p, model, g0, ns, centres, T)
        _compare_eq(y, D.xhi_equilibrium(centres, T, D.gamma_model(model, g0, ns, centres)))
        # denser gas is more neutral (up to rounding once collisions alone set it)
        assert np.all(np.diff(y) >= -4e-16)


@pytest.mark.parametrize("quantity", [rt.HQ_XHI, rt.HQ_GAMMA])
def test_histogram_sums_bit_identical_on_rerun(evolved64, quantity):
    # the per-density-bin sums are exact fixed-point sums rounded once:
    # independent of the order of the additions, so the same state gives the
    # same sums bit for bit
    G, st = evolved64
    yr = (-7.0, 0.5, 64) if quantity == rt.HQ_XHI else (-16.0, -8.0, 64)
    c1, s1 = G.histogram(quantity, (-6.0, 0.0, 48), yr)
    c2, s2 = G.histogram(quantity, (-6.0, 0.0, 48), yr)
    assert np.array_equal(c1, c2)
    assert np.array_equal(s1.view(np.uint64), s2.view(np.uint64))
    assert np.any(s1 != 0.0)


@pytest.mark.parametrize("quantity", [rt.HQ_XHI, rt.HQ_GAMMA])
def test_histogram_sums_are_the_exact_sums(evolved64, quantity):
    # against math.fsum (Shewchuk's exactly rounded summation) of the FP32
    # values per density bin, binned on the FP64 edges: the library sums the
    # FP32 values exactly and rounds once (a few ulp), the rate's sum then
    # scaled by c sigma_n in FP64
    import math

    G, st = evolved64
    nbx, lox, hix = 48, -6.0, 0.0
    yr = (-7.0, 0.5, 64) if quantity == rt.HQ_XHI else (-16.0, -8.0, 64)
    _, sums = G.histogram(quantity, (lox, hix, nbx), yr)
    nH = st["nH"].reshape(-1).astype(np.float64)
    v = (st["xHI"] if quantity == rt.HQ_XHI else st["N"]).reshape(-1)
    edges = np.array([10.0 ** (lox + k * (hix - lox) / nbx) for k in range(nbx + 1)])
    bx = np.clip(np.searchsorted(edges, nH, side="right") - 1, 0, nbx - 1)
    scale = G.params.c_cms * G.params.sigma_n if quantity == rt.HQ_GAMMA else 1.0
    for b in range(nbx):
        ref = math.fsum(v[bx == b].astype(np.float64).tolist())
        ref = ref * scale
        assert abs(sums[b] - ref) <= 4 * np.spacing(abs(ref)), (b, sums[b], ref)
