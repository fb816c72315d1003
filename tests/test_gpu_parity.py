"""Parity of the HIP path (through the C ABI) with the FP64 oracle: one step
from the same FP32-representable state, compared element by element with the
per-field norms of parity_util (N, F <= 1e-4; xHI, T <= 1e-3).

Shapes are chosen to span several 64 x 8 tiles and several z chunks (small
grids take chunks of 8-32 planes) with ragged tails in every axis, every
boundary condition, every chemistry mode, both precisions and both sub-cycle
modes, plus degenerate grids."""

import numpy as np
import pytest

import oracle
from paper_1004_2503_amd import rt
from paper_1004_2503_amd import workloads as W

from parity_util import TOL, assert_parity, errors, one_step_pair

pytestmark = pytest.mark.gpu

DX = 3.0e21
DT = W.courant_dt(DX)
MIXED_BC = (rt.BC_OUTFLOW, rt.BC_REFLECT, rt.BC_PERIODIC, rt.BC_PERIODIC,
            rt.BC_REFLECT, rt.BC_OUTFLOW)


def sources_for(shape, n, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    ijk = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n),
                    rng.integers(0, nz, n)], axis=1).astype(np.int32)
    if n > 1:
        ijk[1] = ijk[0]                          # duplicate cell
    return ijk, 10 ** rng.uniform(50, 53, n)


@pytest.mark.parametrize("chem", [rt.CHEM_FULL, rt.CHEM_ISOTHERMAL, rt.CHEM_OFF,
                                  rt.CHEM_FROZEN])
@pytest.mark.parametrize("prec", [rt.PREC_FP32, rt.PREC_MIXED])
def test_one_step_random_state_ragged(chem, prec):
    shape = (40, 36, 70)
    st = W.random_state(shape, seed=100 + chem)
    src = sources_for(shape, 30, 7)
    g, o, red, _ = one_step_pair(st, shape, DX, DT, 2, MIXED_BC, chem, prec, sources=src)
    e = errors(g, o)
    assert_parity(e, what=f"chem={chem} prec={prec}")
    assert red["n_nonfinite"] == 0


@pytest.mark.parametrize("nsub", [1, 4, 16])
def test_one_step_subcycles(nsub):
    shape = (33, 17, 65)
    st = W.random_state(shape, seed=200 + nsub, nmax=1e-2)
    g, o, red, _ = one_step_pair(st, shape, DX, DT, nsub, (rt.BC_PERIODIC,) * 6,
                                 rt.CHEM_FULL, rt.PREC_MIXED)
    assert_parity(errors(g, o), what=f"nsub={nsub}")


def test_one_step_adaptive_subcycles():
    shape = (20, 24, 66)
    st = W.random_state(shape, seed=300, nmax=1e-2, T_range=(1e2, 3e4))
    g, o, red, og = one_step_pair(st, shape, DX, DT, 64, (rt.BC_OUTFLOW,) * 6,
                                  rt.CHEM_FULL, rt.PREC_MIXED, sub=rt.SUB_ADAPTIVE)
    assert_parity(errors(g, o), what="adaptive")
    hist = np.array(red["subcycle_hist"])
    assert hist.sum() == np.prod(shape)
    assert hist[1:].sum() > 0          # some cells needed more than one sub-cycle
    # total sub-cycles: the histogram brackets the oracle's exact count
    lo = sum(h * (1 << b) for b, h in enumerate(hist))
    hi = sum(h * ((2 << b) - 1) for b, h in enumerate(hist[:7])) + hist[7] * 64
    assert lo * 0.99 <= og.tally[3] <= hi * 1.01


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 1, 1), (1, 1, 7), (1, 9, 1), (3, 4, 65),
                                   (33, 9, 64), (2, 8, 128), (31, 7, 3)])
@pytest.mark.parametrize("bc", [(rt.BC_PERIODIC,) * 6, (rt.BC_OUTFLOW,) * 6,
                                (rt.BC_REFLECT,) * 6])
def test_one_step_degenerate_shapes(shape, bc):
    st = W.random_state(shape, seed=sum(shape) + bc[0])
    src = sources_for(shape, 3, 11)
    g, o, _, _ = one_step_pair(st, shape, DX, DT, 2, bc, rt.CHEM_FULL, rt.PREC_FP32,
                               sources=src)
    assert_parity(errors(g, o), what=f"shape={shape} bc={bc}")


def test_empty_radiation_and_no_sources():
    shape = (9, 10, 11)
    st = W.random_state(shape, seed=5)
    st["N"][...] = 0
    st["Fx"][...] = st["Fy"][...] = st["Fz"][...] = 0
    g, o, red, _ = one_step_pair(st, shape, DX, DT, 1, (rt.BC_PERIODIC,) * 6,
                                 rt.CHEM_FULL, sources=(np.zeros((0, 3), np.int32), []))
    assert np.all(g["N"] == 0)
    assert np.max(np.abs(g["xHI"] - o["xHI"])) <= TOL["xHI"]
    assert np.max(np.abs(g["T"] - o["T"]) / o["T"]) <= TOL["T"]


def test_free_streaming_plane_wave_matches_upwind_closed_form():
    n, steps = 96, 40
    shape = (3, 2, n)
    rng = np.random.default_rng(1)
    N0 = rng.uniform(0.1, 1.0, n).astype(np.float32)
    N = np.broadcast_to(N0, shape).copy()
    st = dict(N=N, Fx=(rt.C_LIGHT * N.astype(np.float64)).astype(np.float32),
              Fy=np.zeros(shape, np.float32), Fz=np.zeros(shape, np.float32),
              xHI=np.ones(shape, np.float32), T=np.full(shape, 1e4, np.float32),
              nH=np.full(shape, 1e-3, np.float32))
    G = rt.RTGrid(rt.make_params(shape, DX, chem=rt.CHEM_OFF), st)
    G.step(DT, 1, steps)
    out = G.state_numpy()
    G.close()
    import math
    want = np.zeros(n)
    for k in range(steps + 1):
        want += math.comb(steps, k) * (1 / 3) ** k * (2 / 3) ** (steps - k) * np.roll(
            N0.astype(np.float64), k)
    assert np.max(np.abs(out["N"][1, 1] - want)) <= 1e-5 * want.max()


def test_reductions_match_oracle_sums():
    shape = (40, 36, 70)
    st = W.random_state(shape, seed=42)
    src = sources_for(shape, 10, 3)
    g, o, red, og = one_step_pair(st, shape, DX, DT, 2, MIXED_BC, rt.CHEM_FULL,
                                  sources=src)
    vol = DX ** 3
    gd = {k: v.astype(np.float64) for k, v in g.items()}
    # FP64 sums of the GPU's own output state
    assert red["xhi_vol"] == pytest.approx(gd["xHI"].mean(), rel=1e-12)
    nh = st["nH"].astype(np.float64)
    assert red["xhi_mass"] == pytest.approx((nh * gd["xHI"]).sum() / nh.sum(), rel=1e-12)
    assert red["photons_stored"] == pytest.approx(gd["N"].sum() * vol, rel=1e-12)
    assert red["gamma_vol"] == pytest.approx(rt.C_LIGHT * rt.SIGMA_N * gd["N"].mean(),
                                             rel=1e-12)
    # and the step tallies against the oracle's
    ro = og.reductions()
    assert red["photons_absorbed"] == pytest.approx(ro["photons_absorbed"], rel=1e-4)
    assert red["photons_escaped"] == pytest.approx(ro["photons_escaped"], rel=1e-4)
    assert red["photons_emitted"] == pytest.approx(ro["photons_emitted"], rel=1e-14)
    assert red["photons_initial"] == pytest.approx(
        st["N"].astype(np.float64).sum() * vol, rel=1e-12)


def test_photon_budget_over_many_steps():
    shape = (48, 40, 72)
    st = W.random_state(shape, seed=9, nH_range=(1e-4, 1e-2))
    G = rt.RTGrid(rt.make_params(shape, DX, bc=MIXED_BC, prec=rt.PREC_MIXED), st)
    G.inject_sources(*sources_for(shape, 40, 2))
    G.step(DT, 2, 100)
    r = G.reduce()
    G.close()
    lhs = r["photons_initial"] + r["photons_emitted"] + r["photons_floor"]
    rhs = r["photons_stored"] + r["photons_absorbed"] + r["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-5)
    assert r["steps"] == 100 and r["n_nonfinite"] == 0


def test_bitwise_deterministic_rerun():
    shape = (40, 36, 70)
    st = W.random_state(shape, seed=77)
    outs = []
    for _ in range(2):
        G = rt.RTGrid(rt.make_params(shape, DX, bc=MIXED_BC, prec=rt.PREC_MIXED), st)
        G.inject_sources(*sources_for(shape, 20, 4))
        G.step(DT, 3, 5)
        outs.append((G.state_numpy(), G.reduce()))
        G.close()
    for k in outs[0][0]:
        assert np.array_equal(outs[0][0][k], outs[1][0][k])
    assert outs[0][1] == outs[1][1]


def test_error_paths_from_the_host():
    shape = (8, 8, 8)
    st = W.random_state(shape, seed=1)
    G = rt.RTGrid(rt.make_params(shape, DX), st)
    assert rt.rt_step(G.ctx, DT * 1.01, 1) == rt.RT_E_CFL
    assert rt.rt_step(G.ctx, DT, 0) == rt.RT_E_ARG
    assert rt.rt_step(G.ctx, -DT, 1) == rt.RT_E_ARG
    assert rt.rt_inject_sources(G.ctx, [[8, 0, 0]], [1e50]) == rt.RT_E_ARG
    assert rt.rt_inject_sources(G.ctx, [[0, 0, 0]], [-1.0]) == rt.RT_E_ARG
    assert rt.rt_inject_sources(G.ctx, [[0, 0, 0]], [float("nan")]) == rt.RT_E_ARG
    assert rt.rt_state(G.ctx, 99, 0x1000, False) == rt.RT_E_ARG
    G.close()
    # a NaN in the input state is reported by rt_reduce
    st2 = {k: v.copy() for k, v in st.items()}
    st2["T"][3, 4, 5] = np.nan
    G = rt.RTGrid(rt.make_params(shape, DX), st2)
    G.step(DT, 1)
    rc, out = rt.rt_reduce(G.ctx)
    assert rc == rt.RT_E_NONFINITE and out.n_nonfinite >= 1
    G.close()


def test_mixed_lf_on_64x8_tiles_with_many_deferred_blocks():
    # Too few 64 x 16 tiles (512) for them to be used, so the LF mixed step
    # runs on 1024 tiles of 64 x 8, and the deferred FP64 chemistry adds 512
    # partial rows after them: 1536 rows, more than either count alone or the
    # state-sum blocks.  Parity, the step's tallies and its FP64 sums.
    shape = (32, 512, 512)
    st = W.random_state(shape, seed=512)
    src = sources_for(shape, 200, 13)
    g, o, red, og = one_step_pair(st, shape, DX, DT, 2, (rt.BC_PERIODIC,) * 6,
                                  rt.CHEM_FULL, rt.PREC_MIXED, sources=src)
    assert_parity(errors(g, o), what="64 x 8 tiles, deferred FP64 chemistry")
    ro = og.reductions()
    assert red["n_fp64"] > 0 and red["n_nonfinite"] == 0
    assert red["photons_absorbed"] == pytest.approx(ro["photons_absorbed"], rel=1e-4)
    assert red["photons_emitted"] == pytest.approx(ro["photons_emitted"], rel=1e-14)
    assert red["xhi_vol"] == pytest.approx(g["xHI"].astype(np.float64).mean(), rel=1e-12)
    vol = DX ** 3
    assert red["photons_stored"] == pytest.approx(g["N"].astype(np.float64).sum() * vol,
                                                  rel=1e-12)


@pytest.mark.parametrize("sub", [rt.SUB_FIXED, rt.SUB_ADAPTIVE])
def test_checkpoint_and_resume_is_bit_identical(sub):
    # Export the state through rt_state after some steps, start a new
    # context from it and continue: every field equals, bit for bit, that of
    # a run that was never interrupted (the step depends only on the state
    # and the sources).
    shape = (40, 36, 70)
    st = W.random_state(shape, seed=505, nmax=1e-2)
    src = sources_for(shape, 25, 12)
    params = rt.make_params(shape, DX, bc=MIXED_BC, prec=rt.PREC_MIXED, sub=sub)
    G = rt.RTGrid(params, st)
    G.inject_sources(*src)
    G.step(DT, 8, 12)
    whole = G.state_numpy()
    G.close()
    G = rt.RTGrid(params, st)
    G.inject_sources(*src)
    G.step(DT, 8, 5)
    ckpt = G.state_numpy()
    G.close()
    R = rt.RTGrid(params, ckpt)
    R.inject_sources(*src)
    R.step(DT, 8, 7)
    resumed = R.state_numpy()
    R.close()
    for k in whole:
        assert np.array_equal(whole[k].view(np.uint32), resumed[k].view(np.uint32)), k


def test_dark_neutral_cells_below_the_temperature_floor():
    # Dark, fully neutral cells skip the chemistry's arithmetic in the step
    # kernel, but the full chemistry still lifts T to T_floor there, as the
    # operator does on every sub-cycle; T below the floor in dark cells (and
    # in lit ones) must come out as the oracle's.
    shape = (20, 18, 66)
    st = W.random_state(shape, seed=606, nmax=1e-3)
    for k in ("N", "Fx", "Fy", "Fz"):
        st[k][:, :, :33] = 0.0
    st["xHI"][:, :, :30] = 1.0
    st["T"][:, :, ::3] = 4.0                       # below the 10 K floor
    for prec in (rt.PREC_FP32, rt.PREC_MIXED):
        g, o, red, _ = one_step_pair(st, shape, DX, DT, 2, (rt.BC_PERIODIC,) * 6,
                                     rt.CHEM_FULL, prec)
        assert_parity(errors(g, o), what=f"T below the floor, prec {prec}")
        dark = (o["N"] == 0) & (st["xHI"] >= 1.0)
        assert dark.any()
        assert np.all(g["T"][dark] >= 10.0)
