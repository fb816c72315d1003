"""Pins of the oracle's M1 closure (Sec. 2.2) against what the mathematics
fixes: the two limits of chi, monotonicity, unit trace of the Eddington
tensor, the isotropic and free-streaming limits and the eigen-structure
(pressure chi*N along the flux, (1-chi)/2*N across it)."""

import numpy as np
import pytest

C = 2.99792458e10


def test_chi_limits(orc):
    assert orc.chi(0.0) == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert orc.chi(1.0) == pytest.approx(1.0, rel=1e-15)


def test_chi_monotone_and_bounded(orc):
    f = np.linspace(0.0, 1.0, 1001)
    chi = np.array([orc.chi(v) for v in f])
    assert np.all(np.diff(chi) > 0)
    assert np.all(chi >= 1.0 / 3.0 - 1e-15) and np.all(chi <= 1.0 + 1e-15)
    # realisability of the 1-D moments: 2f - 1 <= chi, f^2 <= chi
    assert np.all(chi >= f * f - 1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_eddington_trace_and_eigen(orc, seed):
    rng = np.random.default_rng(seed)
    N = 10 ** rng.uniform(-8, 2)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    f = rng.uniform(0.0, 1.0)
    F = d * f * C * N
    P = orc.eddington(N, F, C)
    assert np.allclose(P, P.T)
    assert np.trace(P) == pytest.approx(N, rel=1e-13)
    chi = orc.chi(f)
    assert P @ d == pytest.approx(chi * N * d, rel=1e-12, abs=1e-14 * N)
    perp = np.cross(d, [1.0, 0.0, 0.0])
    perp /= np.linalg.norm(perp)
    assert P @ perp == pytest.approx(0.5 * (1 - chi) * N * perp, rel=1e-12, abs=1e-14 * N)


def test_eddington_isotropic_limit(orc):
    P = orc.eddington(2.5, [0.0, 0.0, 0.0], C)
    assert np.allclose(P, 2.5 * np.eye(3) / 3.0, rtol=1e-15, atol=0)


def test_eddington_free_streaming_limit(orc):
    n = np.array([1.0, -2.0, 2.0]) / 3.0
    P = orc.eddington(4.0, C * 4.0 * n, C)
    assert np.allclose(P, 4.0 * np.outer(n, n), rtol=1e-13, atol=1e-15)


def test_eddington_zero_density(orc):
    assert np.all(orc.eddington(0.0, [0.0, 0.0, 0.0], C) == 0.0)


def test_reduced_flux_clamped(orc):
    # |F| > cN (inadmissible) is treated as free streaming along F
    P = orc.eddington(1.0, [2.0 * C, 0.0, 0.0], C)
    assert np.allclose(P, np.diag([1.0, 0.0, 0.0]), atol=1e-15)
