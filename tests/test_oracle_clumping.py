"""Pins of the oracle's subgrid clumping (Sec. 3.2.1, "Clumping factors"): the
cell-averaged chemistry equation with a recombination clumping factor C_R
on the recombination term and a cross clumping factor C_I on the
photoionisation term, both power laws of the cell density.

  * the factors themselves: C_R = max(1, A_R nH^b_R) (a ratio <y^2>/<y>^2
    cannot be below one), C_I = A_I nH^b_I, and C_R = C_I = 1 when off;
  * clumped photoionisation equilibrium: the closed form with alpha_B nH
    replaced by C_R alpha_B nH and Gamma by C_I Gamma, reached at first
    order in the sub-cycle length (swapping or dropping a factor fails);
  * pure recombination x(t) = x0 / (1 + C_R alpha nH x0 t);
  * collisional-ionisation equilibrium xHI = C_R alpha / (C_R alpha + beta)
    (the collisional term is not clumped), exact at any sub-cycle length;
  * the photo step solves a C_I (nHI - P)(N - P) = P and conserves
    N - nHI;
  * radiative cooling of fully ionised gas (recombination cooling and
    bremsstrahlung, both in ne nHII) scales by C_R;
  * whole method: a Stromgren sphere in uniform clumped gas has
    r_S = (3 Ndot / (4 pi C_R alpha nH^2))^(1/3), t_rec = 1/(C_R alpha nH),
    and the photon budget still closes.

The paper gives the normalisations of its fits only in figures, so the
laws are pinned in form, not in value."""

import numpy as np
import pytest

from test_oracle_stromgren import front_radius_cells

C = 2.99792458e10
SIGMA_N = 2.93e-18
KB = 1.380649e-16


def law_at(nH_ref, C_R, C_I, b_R=0.7, b_I=0.1):
    """Clumping laws with slopes b_R, b_I that take the values C_R, C_I at
    nH_ref."""
    return (C_R / nH_ref ** b_R, b_R, C_I / nH_ref ** b_I, b_I)


def params(orc, chem="ISOTHERMAL", clump=None, shape=(1, 1, 1), dx=1e21, **kw):
    return orc.make_params(shape, dx, chem=getattr(orc, "CHEM_" + chem), clump=clump, **kw)


def test_factors_closed_form_and_clamp(orc):
    cl = (3.0, 0.7, 0.8, 0.2)
    p = params(orc, clump=cl)
    for nH in (1e-6, 1e-4, 1e-2, 1.0, 30.0):
        cr, ci = orc.clumping(p, nH)
        assert cr == pytest.approx(max(1.0, 3.0 * nH ** 0.7), rel=1e-14)
        assert ci == pytest.approx(0.8 * nH ** 0.2, rel=1e-14)
    assert orc.clumping(p, 1e-6)[0] == 1.0      # clamped
    assert orc.clumping(params(orc), 1e-2) == (1.0, 1.0)


def test_unit_factors_reproduce_the_unclumped_operator(orc):
    p0 = params(orc, "FULL")
    p1 = params(orc, "FULL", clump=(1.0, 0.0, 1.0, 0.0))
    args = (3e11, 4, 2e-3, 5e-4, [1e6, -2e5, 3e5], 0.7, 3000.0)
    a, b = orc.chem_cell(p0, *args), orc.chem_cell(p1, *args)
    for u, v in zip(a, b):
        assert np.array_equal(np.asarray(u), np.asarray(v))


def _fixed_point(orc, p, h, N0, nH, T):
    x = 1.0
    for _ in range(200000):
        _, _, xn, _, _, _ = orc.chem_cell(p, h, 1, nH, N0, [0, 0, 0], x, T)
        if abs(xn - x) <= 1e-15 * x:
            return xn
        x = xn
    raise AssertionError("no convergence")


def test_clumped_equilibrium_closed_form(orc):
    nH, T, Gamma = 2e-4, 1e4, 1e-12
    CR, CI = 5.0, 0.5
    p = params(orc, clump=law_at(nH, CR, CI))
    assert orc.clumping(p, nH) == pytest.approx((CR, CI), rel=1e-12)
    N0 = Gamma / (C * SIGMA_N)
    al = CR * orc.rates(T)[0] * nH
    beta = orc.rates(T)[1] * nH
    G = CI * Gamma
    # C_R alpha nH (1-y)^2 = (C_I Gamma + beta (1-y)) y, y = neutral fraction
    a2 = al + beta
    b2 = -(2 * al + G + beta)
    y_eq = (-b2 - np.sqrt(b2 * b2 - 4 * a2 * al)) / (2 * a2)
    # ten times the unclumped worked example's neutral fraction (5.18e-5):
    # C_R / C_I = 10 at this ionisation level
    assert 4.9e-4 < y_eq < 5.3e-4
    errs = []
    for h in (4e9, 2e9, 1e9):
        y = _fixed_point(orc, p, h, N0, nH, T)
        errs.append(abs(y - y_eq) / y_eq)
    assert errs[-1] < 2e-2
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.15), (errs, order)


def test_clumped_recombination_closed_form(orc):
    nH, T, x0, t = 1e-2, 5000.0, 0.9, 2.5e13
    CR = 4.0
    p = params(orc, clump=law_at(nH, CR, 1.0))
    alpha = orc.rates(T)[0]
    exact = x0 / (1 + CR * alpha * nH * x0 * t)
    errs = []
    for nsub in (16, 32, 64, 128):
        _, _, y, _, _, nc = orc.chem_cell(p, t, nsub, nH, 0.0, [0, 0, 0], 1 - x0, T)
        assert nc == nsub
        errs.append(abs((1 - y) - exact) / exact)
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 1.0) < 0.1), (errs, order)
    assert errs[-1] < 1e-2


@pytest.mark.parametrize("CR", [1.0, 6.0])
def test_collisional_ionisation_equilibrium(orc, CR):
    # no radiation: C_R alpha nH x^2 = beta nH x xHI, so xHI = C_R alpha /
    # (C_R alpha + beta); the collisional term carries no clumping factor,
    # and the creation/destruction update has this as its exact fixed point
    nH, T = 1e-3, 2e4
    p = params(orc, clump=law_at(nH, CR, 1.0))
    r = orc.rates(T)
    want = CR * r[0] / (CR * r[0] + r[1])
    assert 0.05 < want < 0.5                 # both processes matter at 2e4 K
    # the closed form maps onto itself, and iterating converges to it
    assert orc.chem_cell(p, 1e13, 1, nH, 0.0, [0, 0, 0], want, T)[2] == pytest.approx(
        want, rel=1e-12)
    x = 0.5
    for _ in range(3000):
        x = orc.chem_cell(p, 1e14, 1, nH, 0.0, [0, 0, 0], x, T)[2]
    assert x == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("CI", [0.3, 2.5])
def test_clumped_photo_step_root(orc, CI):
    N, xHI, nH, h = 2e-2, 0.5, 2e-2, 3e11
    p = params(orc, clump=law_at(nH, 1.0, CI))
    Nout, F, _, _, absorbed, _ = orc.chem_cell(p, h, 1, nH, N, [0.5 * C * N, 0, 0], xHI, 1e4)
    P = N - Nout
    a = CI * C * SIGMA_N * h
    nHI = nH * xHI
    assert absorbed == pytest.approx(P, rel=1e-9)
    assert 0 <= P <= min(N, nHI) * (1 + 1e-12)
    assert abs(a * (nHI - P) * (N - P) - P) <= 1e-9 * max(P, a * nHI * N)
    assert F[0] == pytest.approx(0.5 * C * Nout, rel=1e-12)


def test_clumped_photo_step_conserves_n_minus_nhi(orc):
    N, xHI, nH, h = 3e-6, 0.9, 1e-5, 1e9
    p = params(orc, clump=law_at(nH, 1.0, 3.0))
    Nout, _, xout, _, _, _ = orc.chem_cell(p, h, 1, nH, N, [0, 0, 0], xHI, 1e4)
    assert Nout - nH * xout == pytest.approx(N - nH * xHI, rel=1e-6)
    # C_I = 3 absorbs more than the unclumped step
    N1 = orc.chem_cell(params(orc), h, 1, nH, N, [0, 0, 0], xHI, 1e4)[0]
    assert N - Nout > 2.5 * (N - N1)


def test_ionised_gas_cooling_scales_with_c_r(orc):
    # fully ionised hot gas over a short sub-cycle: the energy lost is h times
    # the ne nHII cooling (recombination + bremsstrahlung); the nHI terms stay
    # negligible because almost nothing recombines within h
    nH, T0, xHI0, h = 1e-2, 1e6, 1e-12, 1e7

    def energy_lost(clump):
        p = params(orc, "FULL", clump=clump)
        _, _, y, T1, _, _ = orc.chem_cell(p, h, 1, nH, 0.0, [0, 0, 0], xHI0, T0)
        e0 = 1.5 * KB * nH * (2.0 - xHI0) * T0
        e1 = 1.5 * KB * nH * (2.0 - y) * T1
        return e0 - e1

    base = energy_lost(None)
    assert base > 0
    for CR in (2.0, 7.0):
        assert energy_lost(law_at(nH, CR, 1.0)) / base == pytest.approx(CR, rel=2e-3)


@pytest.mark.slow
def test_clumped_stromgren_sphere(orc):
    # uniform clumped gas: the closed form with alpha -> C_R alpha; C_I only
    # sharpens the front and leaves the radius unchanged
    ndot, nH, CR = 5e51, 2e-2, 3.0
    alpha = orc.rates(1e4)[0]
    rS = (3.0 * ndot / (4.0 * np.pi * CR * alpha * nH ** 2)) ** (1.0 / 3.0)
    trec = 1.0 / (CR * alpha * nH)
    n = 16
    dx = rS / 10.0                      # r_S = 10 cells
    dt = dx / (3.0 * C)
    bc = (orc.BC_REFLECT, orc.BC_OUTFLOW) * 3
    p = params(orc, clump=law_at(nH, CR, 1.5), shape=(n, n, n), dx=dx, bc=bc)
    g = orc.Grid(p)
    g.set_state(xHI=np.ones((n,) * 3), T=np.full((n,) * 3, 1e4), nH=np.full((n,) * 3, nH))
    g.set_sources(np.zeros((1, 3), np.int32), [ndot / 8.0])
    done = 0
    for frac in (0.5, 1.5):
        s = int(round(frac * trec / dt))
        g.step(dt, 1, s - done)
        done = s
        want = rS * (1.0 - np.exp(-s * dt / trec)) ** (1.0 / 3.0) / dx
        r = front_radius_cells(g, dx)
        assert abs(r - want) < 1.0, (frac, r, want)
    rd = g.reductions()
    lhs = rd["photons_emitted"] + rd["photons_floor"]
    rhs = rd["photons_stored"] + rd["photons_absorbed"] + rd["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-10)
