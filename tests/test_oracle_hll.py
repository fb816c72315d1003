"""Pins of the oracle's HLL flux (Sec. 2.2 names HLL beside LF; the paper's
runs use LF).  The signal speeds are c times the extreme eigenvalues of the
M1 flux Jacobian, evaluated numerically (complex-step Jacobian, numpy
eigenvalues) cell by cell.

  * eigenvalues: isotropic limit +-1/sqrt(3); along the flux the 1-D M1
    system's closed form (chi' +- sqrt(chi'^2 + 4 (chi - f chi'))) / 2;
    free streaming f -> 1 gives both extremes -> mu (cosine of the angle to
    the axis); the mirror symmetry lmin(mu) = -lmax(-mu); causality
    |lambda| <= 1; and the closed form of the extremes from the
    factorisation of the characteristic polynomial,
    (mu chi' +- sqrt(8 (S-1) ((S-1)(1+mu^2) + 1-mu^2) / (3 S^2))) / 2,
    S = sqrt(4 - 3 f^2);
  * the flux: with speeds -c, +c it is the LF flux exactly; a free-streaming
    plane wave is exact upwind (binomial closed form); uniform states stay
    uniform; photons are conserved (periodic); N >= 0 and |F| <= cN at
    Courant 1/3; reflecting walls pass no photons; on small isotropic waves it
    dissipates less than LF."""

import numpy as np
import pytest

from oracle import hll
from paper_1004_2503_amd import workloads as W

from test_oracle_transport import binomial_upwind, load_state

C = 2.99792458e10
DX = 3.0e21
DT = DX / (3 * C)


def chi(f):
    return (3 + 4 * f * f) / (5 + 2 * np.sqrt(4 - 3 * f * f))


def dchi(f, h=1e-6):
    return (chi(f + h) - chi(f - h)) / (2 * h)


def extremes(f, mu, axis=0):
    """Extremes along `axis` for N = 1, F/c at angle acos(mu) to it."""
    f = np.atleast_1d(np.asarray(f, float))
    mu = np.atleast_1d(np.asarray(mu, float))
    F = np.zeros(f.shape + (3,))
    F[..., axis] = f * mu
    F[..., (axis + 1) % 3] = f * np.sqrt(np.clip(1 - mu * mu, 0, 1))
    lam = hll.eigen_extremes(np.ones_like(f), *(C * F[..., k] for k in range(3)), C)
    return lam[..., 2 * axis], lam[..., 2 * axis + 1]


def test_isotropic_limit():
    lo, hi = extremes([1e-9, 1e-7], [0.3, -0.8])
    assert np.allclose(lo, -1 / np.sqrt(3), atol=1e-6)
    assert np.allclose(hi, 1 / np.sqrt(3), atol=1e-6)
    lam = hll.eigen_extremes(np.array([0.0, 1.0]), np.zeros(2), np.zeros(2), np.zeros(2), C)
    assert np.allclose(lam[:, 0::2], -1 / np.sqrt(3)) and np.allclose(lam[:, 1::2], 1 / np.sqrt(3))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_along_the_flux_matches_the_1d_system(axis):
    f = np.array([0.1, 0.4, 0.7, 0.9, 0.99])
    lo, hi = extremes(f, np.ones_like(f), axis)
    c, cp = chi(f), dchi(f)
    disc = np.sqrt(cp * cp + 4 * (c - f * cp))
    assert np.allclose(hi, (cp + disc) / 2, atol=1e-8)
    assert np.allclose(lo, (cp - disc) / 2, atol=1e-8)


def test_free_streaming_and_symmetry_and_causality():
    rng = np.random.default_rng(2)
    mu = rng.uniform(-1, 1, 200)
    lo, hi = extremes(np.full(200, 1 - 1e-12), mu)
    assert np.allclose(lo, mu, atol=1e-5) and np.allclose(hi, mu, atol=1e-5)
    f = rng.uniform(0, 1, 200)
    lo1, hi1 = extremes(f, mu)
    lo2, hi2 = extremes(f, -mu)
    assert np.allclose(lo1, -hi2, atol=1e-12)
    assert np.all(np.abs(lo1) <= 1 + 1e-12) and np.all(np.abs(hi1) <= 1 + 1e-12)
    assert np.all(lo1 <= hi1)


def test_closed_form_of_the_extremes():
    rng = np.random.default_rng(3)
    f = rng.uniform(1e-3, 1 - 1e-9, 2000)
    mu = rng.uniform(-1, 1, 2000)
    lo, hi = extremes(f, mu)
    S = np.sqrt(4 - 3 * f * f)
    Sm1 = 3 * (1 - f * f) / (S + 1)
    K = Sm1 * (1 + mu * mu) + (1 - mu * mu)
    r = np.sqrt(8 * Sm1 * K / (3 * S * S))
    B = mu * dchi(f)
    assert np.allclose(hi, (B + r) / 2, atol=2e-8)
    assert np.allclose(lo, (B - r) / 2, atol=2e-8)


def test_extremes_depend_on_the_reduced_flux_alone():
    # G is homogeneous of degree one in (N, F), so its Jacobian, hence the
    # signal speeds, depend on F/(cN) only: the same reduced fluxes at N
    # from just above the empty threshold to 1e5 give the same extremes,
    # against the closed form.  (A complex step of fixed size, comparable to
    # N near 1e-30, broke this.)
    rng = np.random.default_rng(5)
    f = rng.uniform(1e-3, 1 - 1e-9, 300)
    mu = rng.uniform(-1, 1, 300)
    ref = extremes(f, mu)
    S = np.sqrt(4 - 3 * f * f)
    Sm1 = 3 * (1 - f * f) / (S + 1)
    r = np.sqrt(8 * Sm1 * (Sm1 * (1 + mu * mu) + (1 - mu * mu)) / (3 * S * S))
    B = mu * dchi(f)
    assert np.allclose(ref[1], (B + r) / 2, atol=2e-8)
    for N0 in (1.5e-30, 3e-29, 1e-12, 1e5):
        F = np.zeros(f.shape + (3,))
        F[..., 0] = f * mu
        F[..., 1] = f * np.sqrt(np.clip(1 - mu * mu, 0, 1))
        N = np.full(f.shape, N0)
        lam = hll.eigen_extremes(N, *(C * N * F[..., k] for k in range(3)), C)
        assert np.allclose(lam[:, 0], ref[0], atol=1e-9), N0
        assert np.allclose(lam[:, 1], ref[1], atol=1e-9), N0


def grid(orc, shape, flux, chem=None, bc=(0,) * 6):
    chem = orc.CHEM_OFF if chem is None else chem
    return orc.Grid(orc.make_params(shape, DX, bc=bc, chem=chem, flux=flux))


def test_unit_speeds_give_the_lf_flux(orc):
    import ctypes
    st = W.random_state((6, 7, 9), seed=11)
    g_lf = grid(orc, (6, 7, 9), orc.FLUX_LF, chem=orc.CHEM_FULL)
    g_h = grid(orc, (6, 7, 9), orc.FLUX_HLL, chem=orc.CHEM_FULL)
    load_state(g_lf, st)
    load_state(g_h, st)
    g_lf.step(DT, 2)
    g_h.fill_ghosts()
    lam = np.empty(g_h._U[0].shape + (6,))
    lam[..., 0::2] = -1.0
    lam[..., 1::2] = 1.0
    tl = np.zeros(orc.NTALLY)
    P = ctypes.POINTER(ctypes.c_double)
    ptr = [u.ctypes.data_as(P) for u in g_h._U]
    rc = orc.lib().orc_step_flux(ctypes.byref(g_h.p), DT, 2, *ptr, g_h.xHI.ctypes.data_as(P),
                                 g_h.T.ctypes.data_as(P), g_h.nH.ctypes.data_as(P),
                                 g_h.S.ctypes.data_as(P), np.ascontiguousarray(lam).ctypes.data_as(P),
                                 tl.ctypes.data_as(P))
    assert rc == 0
    for a, b in ((g_lf.N, g_h.N), (g_lf.Fx, g_h.Fx), (g_lf.xHI, g_h.xHI), (g_lf.T, g_h.T)):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [+1, -1])
def test_plane_wave_is_exact_upwind(orc, axis, sign):
    n, steps = 30, 20
    rng = np.random.default_rng(70 + axis)
    N0 = rng.uniform(0.1, 1.0, n)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    g = grid(orc, tuple(shape), orc.FLUX_HLL)
    N = N0.reshape(shape)
    F = [np.zeros(shape) for _ in range(3)]
    F[axis] = sign * C * N
    g.set_state(N=N, Fx=F[0], Fy=F[1], Fz=F[2])
    g.step(DT, 1, steps)
    want = binomial_upwind(N0, steps, sign=sign)
    assert np.max(np.abs(g.N.reshape(-1) - want)) <= 1e-12 * np.max(want)


def test_invariants(orc):
    # uniform stays uniform
    g = grid(orc, (5, 6, 7), orc.FLUX_HLL)
    shp = g.shape
    F = np.array([0.3, -0.2, 0.4]) * C * 1e-3
    g.set_state(N=np.full(shp, 1e-3), Fx=np.full(shp, F[0]), Fy=np.full(shp, F[1]),
                Fz=np.full(shp, F[2]))
    g.step(DT, 1, 2)
    for a in (g.N, g.Fx, g.Fy, g.Fz):
        assert np.allclose(a, a.flat[0], rtol=1e-13, atol=0)
    # photons conserved, positivity and |F| <= cN on a random state
    st = W.random_state((8, 9, 10), seed=4)
    g = grid(orc, (8, 9, 10), orc.FLUX_HLL)
    load_state(g, st)
    n0 = g.N.sum()
    g.step(DT, 1, 3)
    assert g.N.sum() == pytest.approx(n0, rel=1e-12)
    assert g.N.min() >= 0
    Fn = np.sqrt(g.Fx ** 2 + g.Fy ** 2 + g.Fz ** 2)
    assert np.all(Fn <= C * g.N * (1 + 1e-12))


def test_reflecting_walls_pass_no_photons(orc):
    st = W.random_state((7, 6, 8), seed=5)
    g = grid(orc, (7, 6, 8), orc.FLUX_HLL, bc=(2,) * 6)
    load_state(g, st)
    n0 = g.N.sum()
    g.step(DT, 1, 4)
    assert g.N.sum() == pytest.approx(n0, rel=1e-12)


def test_less_diffusive_than_lf_on_isotropic_waves(orc):
    # small perturbations of isotropic radiation obey the linear system with
    # P = N/3, which conserves E = sum (N - <N>)^2 + 3 sum (F/c)^2; numerical
    # dissipation removes E, at speed c/sqrt(3) for HLL against c for LF
    n = 64
    rng = np.random.default_rng(6)
    N0 = (1.0 + 1e-3 * rng.standard_normal(n)).reshape(1, 1, n)
    E = {}
    for flux in (orc.FLUX_LF, orc.FLUX_HLL):
        g = grid(orc, (1, 1, n), flux)
        g.set_state(N=N0, Fx=np.zeros_like(N0), Fy=np.zeros_like(N0), Fz=np.zeros_like(N0))
        g.step(DT, 1, 10)
        E[flux] = np.sum((g.N - g.N.mean()) ** 2) + 3 * np.sum((g.Fx / C) ** 2)
    E0 = np.sum((N0 - N0.mean()) ** 2)
    assert E[orc.FLUX_LF] < E[orc.FLUX_HLL] < E0
