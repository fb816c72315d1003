"""Pins of the oracle's self-shielding models and equilibrium neutral fraction
(Sec. 3.1.5; clumped form Sec. 3.2.1):

  * the models: the plateau is constant; J1 and J4 fall to 1/e of it at their
    characteristic density, J4 as exp(-(nH/n*)^4) (flatter below n*, steeper
    above), both decreasing (the printed exponent of J4 would make it grow);
  * the equilibrium is the fixed point of the oracle's own chemistry operator
    at fixed T and Gamma (independent code: the sub-cycled creation /
    destruction updates), reached at first order in the sub-step and matched
    by its Richardson extrapolation, with and without clumping, in the
    photoionised, the J1 / J4 and the collisional regimes;
  * the worked example nH = 2e-4 cm^-3, T = 1e4 K, Gamma = 1e-12 /s gives
    5.1831e-5 (the value the chemistry pins reach);
  * closed-form limits: no radiation and no collisions -> fully neutral;
    no radiation -> coronal equilibrium alpha/(alpha + beta); strong
    radiation -> C_R alpha nH / (C_I Gamma) at first order;
  * the balance holds to rounding on random inputs, clumped or not;
  * the plateau is the mean rate below the density threshold."""

import math

import numpy as np
import pytest

from oracle import diagnostics as D
from paper_1004_2503_amd import workloads as W

C = 2.99792458e10
SIGMA_N = 2.93e-18
LAW_B = W.CLUMP_LAWS["B"]


def test_models():
    g0, ns = 2e-12, 0.007
    nH = np.array([1e-6, ns / 2, ns, 2 * ns, 0.1])
    assert np.all(D.gamma_model(D.MODEL_UNIFORM, g0, ns, nH) == g0)
    j1 = D.gamma_model(D.MODEL_EXP1, g0, ns, nH)
    j4 = D.gamma_model(D.MODEL_EXP4, g0, ns, nH)
    assert j1[2] == pytest.approx(g0 / math.e, rel=1e-15)
    assert j4[2] == pytest.approx(g0 / math.e, rel=1e-15)
    assert j1[1] == pytest.approx(g0 * math.exp(-0.5), rel=1e-15)
    assert j4[1] == pytest.approx(g0 * math.exp(-1 / 16), rel=1e-15)
    assert j4[3] == pytest.approx(g0 * math.exp(-16), rel=1e-13)
    assert np.all(np.diff(j1) < 0) and np.all(np.diff(j4) < 0)
    assert j4[1] > j1[1] and j4[3] < j1[3]
    assert j1[0] == pytest.approx(g0, rel=1e-3) and j4[0] == pytest.approx(g0, rel=1e-15)


def _params(orc, clump):
    return orc.make_params((1, 1, 1), 1e21, chem=orc.CHEM_ISOTHERMAL, clump=clump)


def _fixed_point(orc, p, h, N0, nH, T):
    y = 0.5      # not 1: fully neutral gas has no electrons to ionise it collisionally
    for _ in range(400000):
        _, _, yn, _, _, _ = orc.chem_cell(p, h, 1, nH, N0, [0, 0, 0], y, T)
        if abs(yn - y) <= 1e-15 * y:
            return yn
        y = yn
    raise AssertionError("no convergence")


@pytest.mark.parametrize("nH,T,gamma,clump", [
    (2e-4, 1e4, 1e-12, None),                                   # photoionised
    (1e-2, 2e4, 3e-13, LAW_B),                                  # clumped
    (0.007, 1.5e4, D.gamma_model(D.MODEL_EXP1, 1e-12, 0.007, 0.007)[()], None),  # J1 at n1*
    (0.009, 1.2e4, D.gamma_model(D.MODEL_EXP4, 1e-12, 0.018, 0.009)[()], LAW_B),  # J4
    (0.05, 2.5e4, 0.0, LAW_B),                                  # collisional only
])
def test_equilibrium_is_the_chemistry_fixed_point(orc, nH, T, gamma, clump):
    # The photon density N0 = Gamma / (c sigma_n) is restored before every
    # sub-step; it stands for a fixed Gamma only while one sub-step absorbs a
    # negligible part of it, i.e. where the equilibrium is photoionised (or
    # without radiation).  Deep in a cutoff the gas would drain the bath.
    p = _params(orc, clump)
    op = p if clump is not None else None
    want = D.xhi_equilibrium(nH, T, gamma, op)[0]
    r = orc.rates(T)
    cr, ci = orc.clumping(p, nH)
    rate = ci * gamma + (cr * r[0] + r[1]) * nH
    h0 = 0.002 / rate
    N0 = gamma / (C * SIGMA_N)
    ys = [_fixed_point(orc, p, h, N0, nH, T) for h in (h0, h0 / 2, h0 / 4)]
    errs = [abs(y - want) / want for y in ys]
    if gamma == 0.0:
        # the creation / destruction update leaves this balance exact at any h
        assert max(errs) < 1e-11, errs
        return
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.15), (errs, order)
    rich = 2 * ys[2] - ys[1]
    assert rich == pytest.approx(want, rel=max(2e-4, 0.05 * errs[2]))


def test_worked_example():
    assert D.xhi_equilibrium(2e-4, 1e4, 1e-12)[0] == pytest.approx(5.1831e-5, rel=2e-4)


def test_closed_form_limits(orc):
    # no radiation, cold gas (no collisions): fully neutral
    assert D.xhi_equilibrium(1e-3, 100.0, 0.0)[0] == 1.0
    # no radiation: coronal equilibrium
    for T in (2e4, 5e4, 1e5):
        a, b = orc.rates(T)[:2]
        assert D.xhi_equilibrium(1e-2, T, 0.0)[0] == pytest.approx(a / (a + b), rel=1e-12)
    # strong radiation: y -> C_R alpha nH / (C_I Gamma)
    p = _params(orc, LAW_B)
    nH, T = 3e-2, 1e4
    cr, ci = orc.clumping(p, nH)
    a = orc.rates(T)[0]
    for g in (1e-6, 1e-8):
        y = D.xhi_equilibrium(nH, T, g, p)[0]
        lead = cr * a * nH / (ci * g)
        assert y == pytest.approx(lead, rel=3 * lead)
        assert abs(y / lead - 1) > 0.0            # a genuine first-order term remains


@pytest.mark.parametrize("clump", [None, LAW_B])
def test_balance_on_random_inputs(orc, clump):
    rng = np.random.default_rng(12)
    n = 400
    nH = 10 ** rng.uniform(-6, 0, n)
    T = 10 ** rng.uniform(2, 5, n)
    g = 10 ** rng.uniform(-18, -10, n)
    g[:40] = 0.0
    p = _params(orc, clump)
    y = D.xhi_equilibrium(nH, T, g, p if clump is not None else None)
    assert np.all((y >= 0) & (y <= 1))
    for i in range(n):
        a, b = orc.rates(T[i])[:2]
        cr, ci = orc.clumping(p, nH[i])
        rec = cr * a * nH[i] * (1 - y[i]) ** 2
        ion = ci * g[i] * y[i] + b * nH[i] * (1 - y[i]) * y[i]
        # 1 - y carries a relative rounding error of ~eps / (1 - y)
        tol = 1e-9 + 4.5e-16 / max(1.0 - y[i], 1e-300)
        assert rec == pytest.approx(ion, rel=tol, abs=1e-300), i


def test_plateau():
    rng = np.random.default_rng(3)
    nH = 10 ** rng.uniform(-6, 0, 10000)
    g = rng.uniform(0.5, 1.5, 10000) * 1e-12
    sel = nH < 1e-3
    assert D.gamma_plateau(nH, g, 1e-3) == pytest.approx(g[sel].mean(), rel=1e-14)
