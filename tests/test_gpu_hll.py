"""GPU parity of the HLL intercell flux (Sec. 2.2 names it beside LF) with
the FP64 oracle, through the C ABI.  The oracle takes its signal speeds from
numerical eigenvalues of the M1 flux Jacobian; the kernel from their closed
form.

  * one fused step from random states on ragged grids spanning several tiles,
    every boundary kind, with sources, chemistry on and off, both
    precisions; the photon tallies (absorbed, escaped) against the oracle's;
  * several steps in a row (the error does not grow beyond FP32 rounding);
  * a free-streaming plane wave along each axis and direction is transported
    by exact upwinding (binomial closed form);
  * photons are conserved between reflecting walls over many steps;
  * the HLL path is really taken (it differs from LF on the same state);
  * the learned chemistry, which runs with LF only, is refused."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_1004_2503_amd import rt
from paper_1004_2503_amd import workloads as W

from parity_util import assert_parity, errors, oracle_grid, oracle_state, one_step_pair

pytestmark = pytest.mark.gpu

DX = 3.0e21
DT = W.courant_dt(DX)
MIXED_BC = (rt.BC_OUTFLOW, rt.BC_REFLECT, rt.BC_PERIODIC, rt.BC_PERIODIC,
            rt.BC_REFLECT, rt.BC_OUTFLOW)
OUTFLOW = (rt.BC_OUTFLOW,) * 6
HLL = rt.FLUX_HLL


def sources_for(shape, n, seed):
    rng = np.random.default_rng(seed)
    ijk = np.stack([rng.integers(0, s, n) for s in shape[::-1]], axis=1).astype(np.int32)
    return ijk, 10 ** rng.uniform(50, 53, n)


@pytest.mark.parametrize("shape", [(40, 36, 70), (9, 70, 130)])
@pytest.mark.parametrize("bc", [(rt.BC_PERIODIC,) * 6, MIXED_BC, OUTFLOW])
def test_one_step_random_state(shape, bc):
    st = W.random_state(shape, seed=500 + shape[0] + bc[0])
    src = sources_for(shape, 20, 4)
    g, o, red, og = one_step_pair(st, shape, DX, DT, 2, bc, rt.CHEM_FULL, sources=src,
                                  flux=HLL)
    e = errors(g, o)
    print(f"HLL shape={shape} bc={bc} errors {e}", flush=True)
    assert_parity(e, what=f"HLL {shape} {bc}")
    ro = og.reductions()
    assert red["photons_absorbed"] == pytest.approx(ro["photons_absorbed"], rel=1e-4)
    if any(b == rt.BC_OUTFLOW for b in bc):
        assert red["photons_escaped"] == pytest.approx(ro["photons_escaped"], rel=1e-4)
    assert red["n_nonfinite"] == 0


@pytest.mark.parametrize("chem,prec", [(rt.CHEM_OFF, rt.PREC_FP32),
                                       (rt.CHEM_ISOTHERMAL, rt.PREC_MIXED),
                                       (rt.CHEM_FULL, rt.PREC_MIXED)])
def test_one_step_chemistry_modes(chem, prec):
    shape = (24, 20, 66)
    st = W.random_state(shape, seed=61 + chem)
    g, o, _, _ = one_step_pair(st, shape, DX, DT, 3, MIXED_BC, chem, prec,
                               sources=sources_for(shape, 10, 5), flux=HLL)
    assert_parity(errors(g, o), what=f"HLL chem={chem} prec={prec}")


def test_several_steps():
    shape = (20, 18, 70)
    st = W.random_state(shape, seed=808, nH_range=(1e-4, 1e-2))
    src = sources_for(shape, 12, 6)
    steps = 6
    G = rt.RTGrid(rt.make_params(shape, DX, bc=MIXED_BC, flux=HLL), st)
    G.inject_sources(*src)
    G.step(DT, 2, steps)
    out = G.state_numpy()
    G.close()
    g = oracle_grid(st, shape, DX, MIXED_BC, oracle.CHEM_FULL, sources=src,
                    flux=oracle.FLUX_HLL)
    g.step(DT, 2, steps)
    e = errors(out, oracle_state(g))
    print(f"HLL {steps} steps errors {e}", flush=True)
    assert_parity(e, what=f"HLL {steps} steps")


def binomial(N0, steps, sign, p=1 / 3):
    want = np.zeros(len(N0))
    for k in range(steps + 1):
        want += math.comb(steps, k) * p ** k * (1 - p) ** (steps - k) * np.roll(N0, sign * k)
    return want


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [+1, -1])
def test_free_streaming_plane_wave_is_exact_upwind(axis, sign):
    n, steps = 70, 30
    rng = np.random.default_rng(90 + axis)
    N0 = rng.uniform(0.1, 1.0, n).astype(np.float32)
    shape = [3, 2, 5]
    shape[2 - axis] = n
    shape = tuple(shape)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    N = np.broadcast_to(N0.reshape(bshape), shape).copy()
    F = [np.zeros(shape, np.float32) for _ in range(3)]
    F[axis] = (sign * rt.C_LIGHT * N.astype(np.float64)).astype(np.float32)
    st = dict(N=N, Fx=F[0], Fy=F[1], Fz=F[2], xHI=np.ones(shape, np.float32),
              T=np.full(shape, 1e4, np.float32), nH=np.full(shape, 1e-3, np.float32))
    G = rt.RTGrid(rt.make_params(shape, DX, chem=rt.CHEM_OFF, flux=HLL), st)
    G.step(DT, 1, steps)
    got = np.moveaxis(G.state_numpy()["N"], 2 - axis, -1)[0, 0].astype(np.float64)
    G.close()
    want = binomial(N0.astype(np.float64), steps, sign)
    err = np.max(np.abs(got - want)) / want.max()
    print(f"plane wave axis={axis} sign={sign}: {err:.2e}", flush=True)
    assert err <= 1e-5


def test_reflecting_box_conserves_photons():
    shape = (30, 26, 68)
    st = W.random_state(shape, seed=31, nH_range=(1e-4, 1e-2))
    G = rt.RTGrid(rt.make_params(shape, DX, bc=(rt.BC_REFLECT,) * 6, chem=rt.CHEM_OFF,
                                 flux=HLL), st)
    G.step(DT, 1, 50)
    r = G.reduce()
    G.close()
    assert r["photons_stored"] == pytest.approx(r["photons_initial"] + r["photons_floor"],
                                                rel=1e-5)
    assert r["photons_escaped"] == 0.0 and r["n_nonfinite"] == 0


def test_hll_differs_from_lf():
    shape = (16, 16, 64)
    st = W.random_state(shape, seed=3)
    outs = []
    for flux in (rt.FLUX_LF, HLL):
        G = rt.RTGrid(rt.make_params(shape, DX, chem=rt.CHEM_OFF, flux=flux), st)
        G.step(DT, 1)
        outs.append(G.state_numpy()["N"].astype(np.float64))
        G.close()
    assert np.max(np.abs(outs[0] - outs[1])) > 1e-2 * np.max(outs[0])


def test_surrogate_runs_with_hll():
    """The learned chemistry runs in the deferred kernel, after either flux:
    with the chemistry off it changes nothing, with it on the HLL step still
    closes the photon budget."""
    shape = (8, 8, 64)
    st = W.random_state(shape, seed=1)
    theta = torch.zeros(rt.MLP_NPARAM, dtype=torch.float32, device="cuda")
    norm = [0.0] * 5 + [1.0] * 5 + [0.0, 0.0, 1.0, 1.0] + [-40.0] * 5 + [40.0] * 5
    outs = []
    for chem in (rt.CHEM_OFF, rt.CHEM_FULL):
        for surr in (False, True):
            G = rt.RTGrid(rt.make_params(shape, DX, flux=HLL, chem=chem), st)
            if surr:
                rt.check(rt.rt_set_surrogate(G.ctx, theta, norm, 1e-2), "rt_set_surrogate")
            G.step(DT, 1)
            red = G.reduce()
            outs.append(G.state_numpy())
            G.close()
            lhs = red["photons_initial"] + red["photons_emitted"] + red["photons_floor"]
            rhs = red["photons_stored"] + red["photons_absorbed"] + red["photons_escaped"]
            assert rhs == pytest.approx(lhs, rel=1e-5)
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_free_streaming_beams_with_vanishing_transverse_speeds(axis):
    # A slab of cells at |F| = cN along one axis (FP32-rounded, so f is 1 to
    # within rounding) with transverse flux components so small that the
    # transverse signal speeds are denormal (~1e-40 in units of c), beside
    # isotropic cells and nearly empty ones (N just above the empty
    # threshold).  Regression: HLL weights formed in units of c took the
    # reciprocal of a denormal a+ - a- there and turned the step to NaN.
    # At f = 1 the flux Jacobian is defective, so the oracle's numerical
    # eigenvalues are ill-conditioned there (errors of order sqrt(rounding));
    # parity is checked on the cells whose stencil does not reach the slab,
    # finiteness, the guards and the photon budget everywhere.
    shape = (20, 24, 66)
    rng = np.random.default_rng(40 + axis)
    N = (1e-3 * rng.random(shape) ** 2 + 1e-8).astype(np.float32)
    c = rt.C_LIGHT
    F = np.zeros((3,) + shape, np.float32)
    beam = np.zeros(shape, bool)
    beam[:, 8:16, :] = True
    F[axis][beam] = (np.float32(c) * N[beam]).astype(np.float32)
    for t in range(3):
        if t != axis:
            F[t][beam] = (1e-40 * c * N[beam].astype(np.float64)
                          * rng.choice([-1.0, 1.0], beam.sum())).astype(np.float32)
    tiny = (rng.random(shape) < 0.05) & ~beam
    N[tiny] = np.float32(1.5e-30)
    F[axis][tiny] = (0.5 * c * N[tiny].astype(np.float64)).astype(np.float32)
    st = dict(N=N, Fx=F[0], Fy=F[1], Fz=F[2],
              xHI=np.full(shape, 0.5, np.float32), T=np.full(shape, 1e4, np.float32),
              nH=np.full(shape, 1e-3, np.float32))
    print(f"HLL vanishing transverse speeds, beams along axis {axis}", flush=True)
    # transport alone (the chemistry would only add a stiff absorber here)
    g, o, red, og = one_step_pair(st, shape, DX, DT, 1, (rt.BC_PERIODIC,) * 6, rt.CHEM_OFF,
                                  flux=HLL)
    assert red["n_nonfinite"] == 0
    for k in ("N", "Fx", "Fy", "Fz", "xHI", "T"):
        assert np.all(np.isfinite(g[k])), k
    assert np.all(g["N"] >= 0.0)
    fl = np.sqrt(g["Fx"].astype(np.float64) ** 2 + g["Fy"].astype(np.float64) ** 2
                 + g["Fz"].astype(np.float64) ** 2)
    assert np.all(fl <= c * g["N"].astype(np.float64) * (1 + 1e-6))
    lhs = red["photons_initial"] + red["photons_emitted"] + red["photons_floor"]
    rhs = red["photons_stored"] + red["photons_absorbed"] + red["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-5)
    near = beam.copy()
    for ax in range(3):
        near |= np.roll(beam, 1, ax) | np.roll(beam, -1, ax)
    far = ~near
    gf = {k: np.where(far, g[k], o[k]) for k in o}
    assert_parity(errors(gf, o), what=f"HLL beams axis {axis}, cells off the slab")
