"""Pins of the oracle's per-cell operator Phi (Appendix A; Sec. 2.2 names
the sub-cycled hydrogen chemistry, the cooling and the gray constants).

  * case-B recombination coefficient at 5000, 10^4 and 2x10^4 K against the
    textbook table (tests/golden/recombination_case_b.txt);
  * the photoionisation step: its absorbed density solves the defining
    backward-Euler relation, lies in [0, min(N, nHI)] and N - nHI is
    conserved by it;
  * photoionisation equilibrium (Sec. 3.1.5 compares its runs with it): under a
    constant photon bath the fixed point tends to the closed-form equilibrium
    at first order in the sub-cycle length;
  * pure recombination: x(t) = x0 / (1 + alpha nH x0 t), first-order
    convergence in the number of sub-cycles;
  * photo-heating with negligible cooling: energy conservation gives the
    final temperature in closed form, with 3.626 eV per ionisation from the
    gray constants of Sec. 2.2;
  * absorption by a frozen neutral density: exp(-c sigma nHI dt) as the
    number of sub-cycles grows;
  * adaptive sub-cycling converges to the fine fixed-step answer."""

import math
import os

import numpy as np
import pytest

C = 2.99792458e10
SIGMA_N = 2.93e-18
KB = 1.380649e-16
EV = 1.602176634e-12
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def params(orc, chem="FULL", sub="FIXED", eps=0.1):
    return orc.make_params((1, 1, 1), 1e21, chem=getattr(orc, "CHEM_" + chem),
                           sub=getattr(orc, "SUB_" + sub), sub_eps=eps)


def test_case_b_recombination_matches_table(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "recombination_case_b.txt"))
    for T, alpha in rows:
        assert orc.rates(T)[0] == pytest.approx(alpha, rel=1e-2)


def test_gray_constants_and_heat_per_ionisation(orc):
    vals = {}
    with open(os.path.join(GOLDEN, "gray_constants.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                vals[line[0]] = float(line[1])
    assert orc.SIGMA_N == vals["sigma_n_cm2"]
    assert orc.SIGMA_E == vals["sigma_e_cm2"]
    assert orc.EGAMMA_EV == vals["egamma_eV"]
    p = params(orc)
    assert orc.heat_per_ionisation_erg(p) / EV == pytest.approx(3.626, abs=5e-4)


def test_rates_positive_and_finite(orc):
    for T in np.logspace(1, 9, 81):
        r = orc.rates(T)
        assert np.all(np.isfinite(r)) and np.all(r >= 0)


@pytest.mark.parametrize("N,xHI,nH,h", [
    (1e-3, 1.0, 2e-4, 1e10),      # photon-rich
    (1e-6, 1.0, 1e-2, 1e12),      # photon-starved
    (5e-3, 1e-4, 1e-2, 1e8),      # nearly ionised
    (2e-2, 0.5, 2e-2, 3e11),      # stiff, comparable densities
])
def test_photoionisation_root(orc, N, xHI, nH, h):
    p = params(orc, "ISOTHERMAL")
    Nout, F, _, _, absorbed, nc = orc.chem_cell(p, h, 1, nH, N, [0.5 * C * N, 0, 0], xHI, 1e4)
    P = N - Nout                       # only the photo step removes photons
    a = C * SIGMA_N * h
    nHI = nH * xHI
    assert absorbed == pytest.approx(P, rel=1e-9, abs=1e-30)
    assert -1e-15 * N <= P <= min(N, nHI) * (1 + 1e-12)
    resid = a * (nHI - P) * (N - P) - P
    assert abs(resid) <= 1e-9 * max(P, a * nHI * N)
    # flux attenuated by the same factor as N
    assert F[0] == pytest.approx(0.5 * C * Nout, rel=1e-12)
    assert nc == 1


def test_photo_step_conserves_n_minus_nhi(orc):
    # with cold, tenuous gas recombination is negligible within h
    p = params(orc, "ISOTHERMAL")
    N, xHI, nH, h = 3e-6, 0.9, 1e-5, 1e9
    Nout, _, xout, _, _, _ = orc.chem_cell(p, h, 1, nH, N, [0, 0, 0], xHI, 1e4)
    assert Nout - nH * xout == pytest.approx(N - nH * xHI, rel=1e-6)


def _equilibrium_fixed_point(orc, h, N0, nH, T):
    p = params(orc, "ISOTHERMAL")
    x = 1.0
    for _ in range(200000):
        _, _, xn, _, _, _ = orc.chem_cell(p, h, 1, nH, N0, [0, 0, 0], x, T)
        if abs(xn - x) <= 1e-15 * x:
            return xn
        x = xn
    raise AssertionError("no convergence")


def test_photoionisation_equilibrium_closed_form(orc):
    nH, T, Gamma = 2e-4, 1e4, 1e-12
    N0 = Gamma / (C * SIGMA_N)
    al = orc.rates(T)[0] * nH
    beta = orc.rates(T)[1] * nH
    # equilibrium of (1-x) Gamma_tot = alpha nH x^2 with collisional term:
    # alpha nH (1-y)^2 = (Gamma + beta (1-y)) y, y = neutral fraction
    a2 = al + beta
    b2 = -(2 * al + Gamma + beta)
    y_eq = (-b2 - np.sqrt(b2 * b2 - 4 * a2 * al)) / (2 * a2)
    # the worked example: nH = 2e-4, T = 1e4 K, Gamma = 1e-12 /s
    assert y_eq == pytest.approx(5.1831e-5, rel=2e-3)
    errs = []
    for h in (4e10, 2e10, 1e10):
        y = _equilibrium_fixed_point(orc, h, N0, nH, T)
        errs.append(abs(y - y_eq) / y_eq)
    assert errs[-1] < 2e-2
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.15), (errs, order)


def test_recombination_closed_form_first_order(orc):
    p = params(orc, "ISOTHERMAL")
    nH, T, x0, t = 1e-2, 5000.0, 0.9, 1e14
    alpha = orc.rates(T)[0]
    exact = x0 / (1 + alpha * nH * x0 * t)
    errs = []
    for nsub in (16, 32, 64, 128):
        _, _, y, _, _, nc = orc.chem_cell(p, t, nsub, nH, 0.0, [0, 0, 0], 1 - x0, T)
        assert nc == nsub
        errs.append(abs((1 - y) - exact) / exact)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.1), (errs, order)
    assert errs[-1] < 1e-2


def test_photoheating_energy_conservation(orc):
    # tenuous neutral gas fully ionised in one sub-cycle: cooling is
    # negligible, so 3/2 kB nH [(1+x1) T1 - (1+x0) T0] = P e_heat
    p = params(orc, "FULL")
    nH, T0, N, h = 1e-10, 100.0, 1.0, 1e10
    Nout, _, y, T1, absorbed, _ = orc.chem_cell(p, h, 1, nH, N, [0, 0, 0], 1.0, T0)
    P = N - Nout
    e_heat = 3.626040955631398 * EV
    x0, x1 = 0.0, 1 - y
    want = ((1 + x0) * T0 + P / nH * e_heat / (1.5 * KB)) / (1 + x1)
    assert T1 == pytest.approx(want, rel=1e-6)
    assert 1.3e4 < T1 < 1.5e4


def test_frozen_absorption_exponential(orc):
    p = params(orc, "FROZEN")
    nH, xHI, N, dt = 1e-3, 0.5, 1e-4, 3e10
    tau = C * SIGMA_N * nH * xHI * dt
    errs = []
    for nsub in (8, 16, 32, 64):
        Nout, _, y, T, _, _ = orc.chem_cell(p, dt, nsub, nH, N, [0, 0, 0], xHI, 1e4)
        assert y == xHI and T == 1e4
        errs.append(abs(Nout - N * np.exp(-tau)) / (N * np.exp(-tau)))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.1)


def test_adaptive_converges_to_fine_fixed(orc):
    nH, N, xHI, T, dt = 1e-2, 3e-3, 1.0, 100.0, 5e11
    ref = orc.chem_cell(params(orc, "FULL"), dt, 20000, nH, N, [0, 0, 0], xHI, T)
    errs = []
    for eps in (0.2, 0.1, 0.05):
        out = orc.chem_cell(params(orc, "FULL", "ADAPTIVE", eps), dt, 100000, nH, N,
                            [0, 0, 0], xHI, T)
        errs.append(abs(out[3] - ref[3]) / ref[3] + abs(out[2] - ref[2]))
        assert out[5] > 1
    assert errs[2] < errs[0]
    assert errs[2] < 2e-2


@pytest.mark.parametrize("ratio", [5.0, 50.0, 500.0])
def test_adaptive_count_for_linear_recombination_growth(orc, ratio):
    # Isothermal ionised gas without photons at 100 K (no collisional
    # ionisation): dxHI/dt = alpha nH (1 - xHI)^2 ~ alpha nH while xHI << 1,
    # so the time over which xHI changes by its own size is xHI/(alpha nH),
    # and sub-steps of eps times it multiply xHI by (1 + eps) each: after k
    # of them t_k = xHI0 ((1 + eps)^k - 1) / (alpha nH).  The step of
    # length dt therefore takes ceil(ln(1 + alpha nH dt / xHI0) / ln(1 + eps))
    # sub-cycles.
    eps, nH, x0, T = 0.1, 1e-3, 1e-6, 100.0
    alpha = orc.rates(T)[0]
    assert orc.rates(T)[1] == 0.0
    dt = ratio * x0 / (alpha * nH)
    out = orc.chem_cell(params(orc, "ISOTHERMAL", "ADAPTIVE", eps), dt, 100000, nH, 0.0,
                        [0, 0, 0], x0, T)
    assert out[5] == math.ceil(math.log(1.0 + ratio) / math.log(1.0 + eps))
    assert out[2] == pytest.approx(x0 * (1.0 + ratio), rel=1e-2)


@pytest.mark.parametrize("T", [3e4, 1e5, 3e5])
def test_adaptive_count_at_coronal_equilibrium(orc, T):
    # At collisional-ionisation equilibrium (no photons, T held) recombination
    # creates neutral hydrogen as fast as collisions destroy it: the net rate
    # is zero, each gross term is alpha nH x^2 (x = 1 - xHI, xHI = alpha /
    # (alpha + beta)).  The state does not move, and a controller on the
    # gross rate takes sub-steps of eps xHI / (2 alpha nH x^2) throughout:
    # ceil(dt / that) sub-cycles (one on the net rate).
    eps, nH = 0.1, 1e-3
    a, b = orc.rates(T)[:2]
    xe = a / (a + b)
    x = 1.0 - xe
    h = eps * xe / (2.0 * a * nH * x * x)
    dt = 37.3 * h
    out = orc.chem_cell(params(orc, "ISOTHERMAL", "ADAPTIVE", eps), dt, 100000, nH, 0.0,
                        [0, 0, 0], xe, T)
    assert out[5] == math.ceil(dt / h)
    assert out[2] == pytest.approx(xe, rel=1e-12)


def test_adaptive_cap_and_time_coverage(orc):
    # with the cap reached the last sub-cycle takes what remains of dt; the
    # result is then identical to taking a single remaining step
    p = params(orc, "FULL", "ADAPTIVE", 0.1)
    out = orc.chem_cell(p, 1e12, 3, 1e-2, 3e-3, [0, 0, 0], 1.0, 100.0)
    assert out[5] == 3


def test_xhi_and_temperature_floors(orc):
    p = params(orc, "FULL")
    # enormous photon density ionises everything: xHI hits its floor
    out = orc.chem_cell(p, 1e12, 1, 1e-6, 1e3, [0, 0, 0], 1.0, 1e4)
    assert out[2] >= 1e-12
    # dense cold gas cools to the floor
    out = orc.chem_cell(p, 1e16, 4, 10.0, 0.0, [0, 0, 0], 1e-3, 12.0)
    assert out[3] >= 10.0
