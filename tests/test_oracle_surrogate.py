"""Pins of the oracle's learned-chemistry arithmetic (oracle/surrogate.py):
photon accounting, the backward-Euler acceptance test and the fallback
conditions.  Not part of the paper; the reading is the one in the module
docstring.

  * the photon budget closes exactly: N' + P = N~, P in [0, N~], F scaled
    like N;
  * the residuals vanish at the end point of one backward-Euler step of the
    chemistry ODEs of Sec. 2.2 (photoionisation, case-B recombination and
    collisional ionisation, photo-heating and cooling), found here by a
    root finder from the ODE right-hand sides, and grow when that end point
    is perturbed;
  * out-of-range features, bounds violations and non-full chemistry fall
    back;
  * plausible mistakes planted in the accounting's inputs (a rate off by a
    factor, the clumping factors swapped) break the backward-Euler pin.
"""

import numpy as np
import pytest
from scipy import optimize

import oracle
from oracle import mlp
from oracle import surrogate as S

KB = 1.380649e-16
DX = 3.0e21


def params(chem=oracle.CHEM_FULL, clump=None):
    return oracle.make_params((1, 1, 1), DX, chem=chem, clump=clump)


def be_end_point(p, dt, nH, Nt, xHI, T, rates=oracle.rates):
    """End point (N', xHI', T') of one backward-Euler step of length dt of
    dN/dt = -C_I c sigma_n N nHI, dnHI/dt = -C_I c sigma_n N nHI +
    C_R alpha_B ne nHII - beta ne nHI, du/dt = C_I c sigma_n N nHI e_heat -
    Lambda, with u = 3/2 kB nH (1 + x) T, written from those right-hand
    sides and solved by a root finder (log variables keep it positive)."""
    CR, CI = oracle.clumping(p, nH)
    g = CI * p.c * p.sigma_n
    eh = oracle.heat_per_ionisation_erg(p)

    def resid(v):
        xs, Ts = np.exp(v[0]), np.exp(v[1])
        x1 = 1.0 - xs
        r = rates(Ts)
        Ne = Nt / (1.0 + dt * g * nH * xs)
        ion = g * Ne * nH * xs
        f1 = nH * (xs - xHI) - dt * (-ion + CR * r[0] * nH * nH * x1 * x1 -
                                     r[1] * nH * nH * x1 * xs)
        lam = CR * nH * nH * x1 * x1 * (r[2] + r[5]) + nH * nH * x1 * xs * (r[3] + r[4])
        f2 = 1.5 * KB * nH * ((1.0 + x1) * Ts - (1.0 + (1.0 - xHI)) * T) - dt * (ion * eh - lam)
        return [f1 / (nH * xHI + 1e-300), f2 / (1.5 * KB * nH * T)]

    # start from the exact operator's answer
    _, _, x_g, T_g, _, _ = oracle.chem_cell(p, dt, 32, nH, Nt, (0.0, 0.0, 0.0), xHI, T)
    sol = optimize.root(resid, [np.log(max(x_g, 1e-12)), np.log(T_g)], method="hybr",
                        options=dict(xtol=1e-14))
    # (hybr may stop at rounding level with "no further improvement")
    assert max(abs(v) for v in resid(sol.x)) < 1e-10, sol
    xs, Ts = np.exp(sol.x)
    Ne = Nt / (1.0 + dt * CI * p.c * p.sigma_n * nH * xs)
    return Ne, xs, Ts


CELLS = [
    # nH [cm^-3], N~ [cm^-3], xHI, T [K], dt [s]
    (2e-4, 1e-6, 0.999, 1e4, 1e11),
    (1e-3, 3e-5, 0.5, 2e4, 3e11),
    (5e-2, 1e-4, 0.99, 8e3, 2e11),
    (1e-4, 1e-9, 1e-4, 3e4, 4e11),
    (3e-3, 2e-7, 0.1, 1.5e4, 1e12),
]


def _acc(p, dt, nH, Nt, xHI, T, xs, Ts, tol=1e-3, ood=False, F=(0.0, 0.0, 0.0), **kw):
    return S.accounting(p, dt, [nH], [Nt], [F[0]], [F[1]], [F[2]], [xHI], [T], [xs], [Ts],
                        tol, [ood], **kw)


def test_budget_closes_exactly_for_any_prediction():
    p = params()
    rng = np.random.default_rng(5)
    n = 2000
    nH = 10 ** rng.uniform(-5, -1, n)
    Nt = 10 ** rng.uniform(-12, -3, n)
    xHI = 10 ** rng.uniform(-6, 0, n)
    T = 10 ** rng.uniform(2, 4.7, n)
    xs = np.clip(xHI * 10 ** rng.uniform(-3, 1, n), 1e-12, 1.0)
    Ts = T * 10 ** rng.uniform(-0.5, 0.5, n)
    F = [Nt * p.c * rng.uniform(-0.5, 0.5, n) for _ in range(3)]
    a = S.accounting(p, 1e11, nH, Nt, *F, xHI, T, xs, Ts, 1e-3, np.zeros(n, bool))
    assert np.all(a["P"] >= 0.0) and np.all(a["P"] <= Nt)
    assert np.all(a["N"] >= 0.0)
    assert np.all(np.abs(a["N"] + a["P"] - Nt) <= 1e-15 * Nt)
    for k, Fk in zip(("Fx", "Fy", "Fz"), F):
        assert np.allclose(a[k], Fk * a["N"] / Nt, rtol=1e-14, atol=0.0)
    # the photons absorbed are the implied net ionisations where no clamp acts
    r = oracle.rates_n(Ts)
    x1 = 1.0 - xs
    raw = nH * (xHI - xs) + r[:, 0] * nH * nH * x1 * x1 * 1e11 - r[:, 1] * nH * nH * x1 * xs * 1e11
    free = (raw > 0) & (raw < Nt)
    assert free.sum() > 100
    assert np.allclose(a["P"][free], raw[free], rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("clump", [None, (30.0, 0.7, 2.0, 0.15)])
@pytest.mark.parametrize("cell", CELLS)
def test_residuals_vanish_at_the_backward_euler_end_point(cell, clump):
    p = params(clump=clump)
    nH, Nt, xHI, T, dt = cell
    Ne, xs, Ts = be_end_point(p, dt, nH, Nt, xHI, T)
    a = _acc(p, dt, nH, Nt, xHI, T, xs, Ts)
    assert a["rx"][0] <= 1e-9 * xs and a["rT"][0] <= 1e-9, (a["rx"], a["rT"])
    assert a["N"][0] == pytest.approx(Ne, rel=1e-9, abs=1e-9 * Nt)
    assert a["ok"][0]
    # a prediction 5e-3 off the end point in xHI (the residual of xHI is
    # absolute, like the xHI parity norm) or 5% off in T is rejected at 1e-4
    assert not _acc(p, dt, nH, Nt, xHI, T, xs, Ts * 1.05, tol=1e-4)["ok"][0]
    if xs > 1e-2:
        assert not _acc(p, dt, nH, Nt, xHI, T, xs - 5e-3, Ts, tol=1e-4)["ok"][0]


def test_fallback_conditions():
    p = params()
    nH, Nt, xHI, T, dt = CELLS[0]
    _, xs, Ts = be_end_point(p, dt, nH, Nt, xHI, T)
    assert _acc(p, dt, nH, Nt, xHI, T, xs, Ts)["ok"][0]
    assert not _acc(p, dt, nH, Nt, xHI, T, xs, Ts, ood=True)["ok"][0]
    assert not _acc(p, dt, nH, Nt, xHI, T, 1.0 + 1e-6, Ts, tol=1.0)["ok"][0]
    assert not _acc(p, dt, nH, Nt, xHI, T, 1e-13, Ts, tol=1.0)["ok"][0]
    assert not _acc(p, dt, nH, Nt, xHI, T, xs, 0.5 * p.T_floor, tol=1e9)["ok"][0]
    assert not _acc(p, dt, nH, Nt, xHI, T, xs, np.nan, tol=1e9)["ok"][0]
    assert not _acc(p, dt, nH, Nt, xHI, T, xs, np.inf, tol=1e9)["ok"][0]
    for chem in (oracle.CHEM_ISOTHERMAL, oracle.CHEM_OFF, oracle.CHEM_FROZEN):
        assert not _acc(params(chem=chem), dt, nH, Nt, xHI, T, xs, Ts, tol=1e9)["ok"][0]


def test_features_decode_and_range():
    f = S.features([2e-4, 1.0], [0.0, 1e-5], [1.0, 1e-40], [1e4, 3e4], 1e11)
    assert f[0, 3] == pytest.approx(-30.0) and f[1, 1] == pytest.approx(-30.0)
    assert f[0, 0] == pytest.approx(np.log10(2e-4)) and f[1, 4] == pytest.approx(11.0)
    norm = np.concatenate([np.zeros(5), np.ones(5), [0.0, 0.0], [1.0, 1.0],
                           np.full(5, -40.0), np.full(5, 40.0)])
    # zero output = no change: u = 0 decodes to d = 0
    xs, Ts = S.decode(f, np.zeros((2, 2)), norm)
    assert np.allclose(xs, [1.0, 1e-30], rtol=1e-13) and np.allclose(Ts, [1e4, 3e4], rtol=1e-13)
    # u = asinh(d / 1e-3) inverts exactly
    d = np.array([[0.3, -0.01], [-2.0, 1e-5]])
    xs, Ts = S.decode(f, np.arcsinh(d / 1e-3), norm)
    assert np.allclose(np.log10(xs) - f[:, 1], d[:, 0], rtol=1e-12, atol=1e-14)
    assert np.allclose(np.log10(Ts) - f[:, 2], d[:, 1], rtol=1e-12, atol=1e-14)
    assert not S.out_of_range(f, norm).any()
    bad = f.copy()
    bad[0, 2] = 41.0
    bad[1, 0] = np.nan
    assert S.out_of_range(bad, norm).all()


def test_constant_network_outputs_its_bias():
    theta = mlp.init_params(3)
    off = sum(o * i + o for o, i in mlp.SIZES[:-1])
    theta[off:off + 128] = 0.0              # W4 = 0
    theta[off + 128:off + 130] = [0.25, -1.5]
    norm = np.concatenate([np.zeros(5), np.ones(5), np.zeros(4), np.full(5, -50),
                           np.full(5, 50)])
    f = np.random.default_rng(0).normal(size=(50, 5))
    y = S.network_outputs(theta, norm, f)
    assert np.array_equal(y, np.tile([0.25, -1.5], (50, 1)))


def test_planted_mistakes_break_the_backward_euler_pin():
    nH, Nt, xHI, T, dt = CELLS[1]

    def alpha_doubled(Tv):
        r = oracle.rates_n(Tv)
        r[:, 0] *= 2.0
        return r

    def cooling_tenfold(Tv):
        r = oracle.rates_n(Tv)
        r[:, 3] *= 10.0
        return r

    p = params()
    _, xs, Ts = be_end_point(p, dt, nH, Nt, xHI, T)
    for rates in (alpha_doubled, cooling_tenfold):
        a = _acc(p, dt, nH, Nt, xHI, T, xs, Ts, tol=1e-6, rates=rates)
        assert not a["ok"][0], rates.__name__
    pc = params(clump=(30.0, 0.7, 2.0, 0.15))
    _, xs, Ts = be_end_point(pc, dt, nH, Nt, xHI, T)

    def swapped(q, n):
        cr, ci = oracle.clumping(q, n)
        return ci, cr

    a = _acc(pc, dt, nH, Nt, xHI, T, xs, Ts, tol=1e-6, clump=swapped)
    assert not a["ok"][0]
