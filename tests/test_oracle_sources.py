"""Pins of the oracle's source pipeline (Sec. 2.3: lifetimes, snapshot
dilution, escape fraction and boost factor, nearest-grid-point projection).

  * the three cases the paper lists for a particle of snapshot p+1: dead
    before t_p (discarded), born within the interval (emits for its age),
    alive at t_p (emits until the interval ends or its lifetime does);
  * photon conservation: over consecutive snapshot intervals, any spacing, a
    particle emits exactly Q m / m_b photons in total, its lifetime output;
  * the boost factor with the paper's table values (100 Mpc/h box: a_b 1.2,
    k_b 3000 Myr) is e^3 * 1.2 at t = 1 Gyr and never below one;
  * NGP: positions in a cell map to it, the periodic box wraps, duplicate
    cells sum, and the field holds every emitted photon."""

import numpy as np
import pytest

from oracle import sources as S

MYR = S.MYR


def test_three_cases_of_the_interval():
    delta = 2.0 * MYR
    L = 10.0 * MYR
    # dead before t_p: a_p = 13 - 2 = 11 Myr >= L
    assert S.emitting_overlap(13 * MYR, L, delta) == 0.0
    # born within the interval: a_p < 0, emits for its age 1.5 Myr
    assert S.emitting_overlap(1.5 * MYR, L, delta) == pytest.approx(1.5 * MYR, rel=1e-15)
    # alive at t_p and through the interval
    assert S.emitting_overlap(5 * MYR, L, delta) == pytest.approx(2 * MYR, rel=1e-15)
    # alive at t_p, dies within: min(delta, L - a_p) = 10 - 9.5 = 0.5 Myr
    assert S.emitting_overlap(11.5 * MYR, L, delta) == pytest.approx(0.5 * MYR, rel=1e-12)
    # born and dead within the interval (L shorter than the interval)
    assert S.emitting_overlap(3 * MYR, 1 * MYR, 4 * MYR) == pytest.approx(1 * MYR, rel=1e-15)


def test_lifetime_photons_conserved_over_snapshots():
    rng = np.random.default_rng(1)
    n = 500
    L = rng.uniform(5, 20, n) * MYR
    Q = rng.uniform(24000, 98000, n)
    m = rng.uniform(1e37, 1e38, n)
    birth = rng.uniform(0, 30, n) * MYR
    for spacing in (0.7, 3.0, 11.0):
        edges = np.arange(0.0, 60.0 + spacing, spacing) * MYR
        total = np.zeros(n)
        for t0, t1 in zip(edges[:-1], edges[1:]):
            age_next = t1 - birth
            alive = age_next >= 0              # in snapshot p+1 only once born
            r = S.particle_rates(age_next, L, Q, m, t0, t1, 1.0, 0.0, 1.0)
            total += np.where(alive, r, 0.0) * (t1 - t0)
        assert np.allclose(total, Q * m / S.M_BARYON, rtol=1e-12), spacing


def test_boost_factor_table_values():
    a_b, k_b = 1.2, 3000 * MYR
    assert S.boost(1000 * MYR, a_b, k_b) == pytest.approx(1.2 * np.exp(3.0), rel=1e-14)
    # the 12.5 Mpc/h box (a_b 0.7, k_b 300 Myr) late on: no boost below one
    assert S.boost(1e4 * MYR, 0.7, 300 * MYR) == 1.0
    assert S.boost(50 * MYR, 0.7, 300 * MYR) == pytest.approx(0.7 * np.exp(6.0), rel=1e-14)


def test_effective_rate_factors():
    # interval 999 - 1001 Myr: the boost is taken at 1000 Myr
    r = S.particle_rates(5 * MYR, 10 * MYR, 50000.0, 2e38, 999 * MYR, 1001 * MYR, 0.03, 1.2,
                         3000 * MYR)
    Ndot = 50000.0 * 2e38 / S.M_BARYON / (10 * MYR)
    want = Ndot * 0.03 * 1.2 * np.exp(3.0)
    assert np.isfinite(r) and r == pytest.approx(want, rel=1e-12)


def test_ngp_wrap_and_sum():
    dx = 2.0
    shape = (4, 3, 5)                           # nz, ny, nx
    pos = np.array([[0.1, 0.1, 0.1], [1.99, 5.9, 7.99], [10.0, 6.0, 8.0],
                    [-0.5, -0.5, -0.5], [0.3, 0.2, 0.1]])
    ijk = S.ngp_cells(pos, dx, shape)
    assert ijk.tolist() == [[0, 0, 0], [0, 2, 3], [0, 0, 0], [4, 2, 3], [0, 0, 0]]
    F = S.source_field(ijk, [1.0, 2.0, 4.0, 8.0, 16.0], shape)
    assert F[0, 0, 0] == 21.0 and F[3, 2, 0] == 2.0 and F[3, 2, 4] == 8.0
    assert F.sum() == 31.0
