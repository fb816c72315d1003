"""Whole-method pin of the oracle: a point source in uniform isothermal
(10^4 K) hydrogen grows an ionised sphere whose radius follows the
closed form r_I(t) = r_S (1 - exp(-t/t_rec))^(1/3), with the Stromgren radius
r_S = (3 Ndot / (4 pi alpha_B nH^2))^(1/3) and t_rec = 1/(alpha_B nH).

The source sits in the corner cell; the three faces meeting there reflect
and the rest are outflow, so the grid holds one octant of the sphere and the
injected rate is Ndot/8.  r_I is the volume-equivalent radius of the octant,
(6 V / pi)^(1/3) with V = sum (1 - xHI) dx^3.  Pass: within one cell.

Two set-ups: the 32^3 configuration itself (weak: the front has moved ~2
cells after 500 steps) and a brighter, denser 16^3 variant in which the front
travels ~10 cells (0.25 and 1 recombination time)."""

import numpy as np
import pytest

from paper_1004_2503_amd import workloads as W

C = 2.99792458e10


def front_radius_cells(g, dx):
    V = float(np.sum(1.0 - g.xHI)) * dx ** 3
    return (6.0 * V / np.pi) ** (1.0 / 3.0) / dx


def closed_form(orc, ndot, nH, t, T=1e4):
    alpha = orc.rates(T)[0]
    rS = (3.0 * ndot / (4.0 * np.pi * alpha * nH ** 2)) ** (1.0 / 3.0)
    trec = 1.0 / (alpha * nH)
    return rS * (1.0 - np.exp(-t / trec)) ** (1.0 / 3.0), rS, trec


def run(orc, n, dx, dt, ndot, nH, steps_list):
    bc = (orc.BC_REFLECT, orc.BC_OUTFLOW) * 3
    p = orc.make_params((n, n, n), dx, bc=bc, chem=orc.CHEM_ISOTHERMAL)
    g = orc.Grid(p)
    g.set_state(xHI=np.ones((n,) * 3), T=np.full((n,) * 3, 1e4),
                nH=np.full((n,) * 3, nH))
    g.set_sources(np.zeros((1, 3), np.int32), [ndot / 8.0])
    out, done = [], 0
    for s in steps_list:
        g.step(dt, 1, s - done)
        done = s
        out.append(front_radius_cells(g, dx))
    return g, out


def test_stromgren_config_32(orc):
    w = W.workload("stromgren32")
    ndot, nH = w.extra["ndot"], w.nH_mean
    _, radii = run(orc, 32, w.dx, w.dt, ndot, nH, [200, 500])
    for steps, r in zip([200, 500], radii):
        want, rS, _ = closed_form(orc, ndot, nH, steps * w.dt)
        assert rS / w.dx == pytest.approx(16.47, rel=2e-3)
        assert abs(r - want / w.dx) < 1.0, (steps, r, want / w.dx)


@pytest.mark.slow
def test_stromgren_fast_variant(orc):
    ndot, nH = 5e51, 2e-2
    _, rS, trec = closed_form(orc, ndot, nH, 1.0)
    dx = rS / 12.0                      # r_S = 12 cells
    dt = W.courant_dt(dx)
    steps = [int(round(0.25 * trec / dt)), int(round(trec / dt))]
    g, radii = run(orc, 16, dx, dt, ndot, nH, steps)
    for s, r in zip(steps, radii):
        want = closed_form(orc, ndot, nH, s * dt)[0] / dx
        assert abs(r - want) < 1.0, (s, r, want)
    # the photon budget closes over the whole run
    rd = g.reductions()
    lhs = rd["photons_emitted"] + rd["photons_floor"]
    rhs = rd["photons_stored"] + rd["photons_absorbed"] + rd["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-10)
