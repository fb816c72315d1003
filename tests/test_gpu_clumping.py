"""GPU parity of the subgrid clumping model (Sec. 3.2.1, clumping factors) with
the FP64 oracle, through the C ABI:

  * the batch operator rt_chem_apply with the 'B' laws (C_R ~ nH^0.7,
    C_I ~ nH^0.1) and the 'A' laws (C_R ~ nH^2.5, C_I = 1), every chemistry
    mode, both precisions, fixed and adaptive sub-cycling, cell by cell;
  * one fused step from a random state on a ragged grid that spans several
    tiles, with sources and mixed boundaries;
  * unit laws (norms 1, slopes 0) give results bit-identical to the
    unclumped path;
  * a clumped 128^3 cosmological run: one step from the library's evolved
    state against the oracle everywhere, and the photon budget of the run.

The laws' normalisations are the paper's shapes with values chosen here
(the paper shows them only in figures)."""

import numpy as np
import pytest
import torch

import oracle
from paper_1004_2503_amd import rt
from paper_1004_2503_amd import workloads as W

from parity_util import assert_parity, errors, oracle_grid, oracle_state, one_step_pair

pytestmark = pytest.mark.gpu

DEV = "cuda"
# 'B' laws: C_R from 1 (nH <~ 4e-3) to ~10 at 0.1 cm^-3; C_I 0.7 - 1.8
LAW_B = W.CLUMP_LAWS["B"]
# 'A' laws: C_R ~ nH^2.5 above ~0.025 cm^-3 (31 at 0.1), C_I = 1
LAW_A = W.CLUMP_LAWS["A"]
MIXED_BC = (rt.BC_OUTFLOW, rt.BC_REFLECT, rt.BC_PERIODIC, rt.BC_PERIODIC,
            rt.BC_REFLECT, rt.BC_OUTFLOW)


def cells(n, seed):
    rng = np.random.default_rng(seed)
    nH = 10 ** rng.uniform(-5, -0.5, n)
    N = 10 ** rng.uniform(-9, -2, n)
    N[: n // 10] = 0.0
    xHI = 10 ** rng.uniform(-6, 0, n)
    T = 10 ** rng.uniform(1.5, 4.8, n)
    dt = 10 ** rng.uniform(9, 12.5, n)
    return [a.astype(np.float32) for a in (nH, N, xHI, T, dt)]


@pytest.mark.parametrize("law", ["B", "A"])
@pytest.mark.parametrize("chem", ["FULL", "ISOTHERMAL", "FROZEN"])
@pytest.mark.parametrize("prec,sub,nsub", [("FP32", "FIXED", 4), ("MIXED", "FIXED", 1),
                                           ("MIXED", "ADAPTIVE", 32)])
def test_chem_apply_clumped_matches_oracle(law, chem, prec, sub, nsub):
    cl = LAW_B if law == "B" else LAW_A
    n = 3000
    nH, N, xHI, T, dt = cells(n, 23)
    p = rt.make_params((1, 1, 1), 1e21, chem=getattr(rt, "CHEM_" + chem),
                       prec=getattr(rt, "PREC_" + prec), sub=getattr(rt, "SUB_" + sub),
                       clump=cl)
    t = [torch.tensor(a, device=DEV) for a in (nH, N, xHI, T, dt)]
    rt.check(rt.rt_chem_apply(p, t[0], t[1], t[2], t[3], t[4], nsub), "rt_chem_apply")
    torch.cuda.synchronize()
    gN, gx, gT = (a.cpu().numpy().astype(np.float64) for a in t[1:4])
    op = oracle.make_params((1, 1, 1), 1e21, chem=getattr(oracle, "CHEM_" + chem),
                            sub=getattr(oracle, "SUB_" + sub), clump=cl)
    errs = np.zeros((n, 3))
    crs = np.zeros(n)
    for i in range(n):
        oN, _, ox, oT, _, _ = oracle.chem_cell(op, float(dt[i]), nsub, float(nH[i]),
                                               float(N[i]), [0, 0, 0], float(xHI[i]),
                                               float(T[i]))
        errs[i] = [abs(gN[i] - oN) / max(float(N[i]), 1e-30), abs(gx[i] - ox),
                   abs(gT[i] - oT) / oT]
        crs[i] = oracle.clumping(op, float(nH[i]))[0]
    worst = errs.max(axis=0)
    if not (worst[0] <= 1e-4 and worst[1] <= 1e-3 and worst[2] <= 1e-3):
        for f in range(3):                       # name the worst cells
            i = int(np.argmax(errs[:, f]))
            print(f"field {f}: cell {i} nH={nH[i]:.6e} N={N[i]:.6e} xHI={xHI[i]:.6e} "
                  f"T={T[i]:.6e} dt={dt[i]:.6e} C_R={crs[i]:.4g} | gpu N={gN[i]:.6e} "
                  f"x={gx[i]:.6e} T={gT[i]:.6e}", flush=True)
    assert worst[0] <= 1e-4 and worst[1] <= 1e-3 and worst[2] <= 1e-3, worst
    # the laws are exercised: a spread of C_R above one
    assert crs.max() > 5.0 and np.mean(crs > 1.0) > 0.05


@pytest.mark.parametrize("chem", [rt.CHEM_FULL, rt.CHEM_ISOTHERMAL])
@pytest.mark.parametrize("prec", [rt.PREC_FP32, rt.PREC_MIXED])
def test_one_step_clumped_random_state(chem, prec):
    shape = (40, 36, 70)
    st = W.random_state(shape, seed=400 + chem, nH_range=(1e-5, 3e-1))
    rng = np.random.default_rng(8)
    ijk = np.stack([rng.integers(0, s, 25) for s in shape[::-1]], axis=1).astype(np.int32)
    src = (ijk, 10 ** rng.uniform(50, 53, 25))
    dx = 3.0e21
    g, o, red, _ = one_step_pair(st, shape, dx, W.courant_dt(dx), 3, MIXED_BC, chem, prec,
                                 sources=src, clump=LAW_B)
    assert_parity(errors(g, o), what=f"clumped chem={chem} prec={prec}")
    assert red["n_nonfinite"] == 0


def test_unit_laws_are_bitwise_unclumped():
    shape = (24, 20, 66)
    st = W.random_state(shape, seed=77)
    dx = 3.0e21
    outs = []
    for cl in (None, (1.0, 0.0, 1.0, 0.0)):
        G = rt.RTGrid(rt.make_params(shape, dx, prec=rt.PREC_MIXED, clump=cl), st)
        G.step(W.courant_dt(dx), 2, 3)
        outs.append(G.state_numpy())
        G.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_clumped_cosmological_run():
    w = W.workload("cosmo128")
    nH, ijk, ndot = W.cosmo_inputs(w, device=DEV)
    shape = (w.n,) * 3
    G = rt.RTGrid(rt.make_params(shape, w.dx, prec=rt.PREC_MIXED, clump=LAW_B), dict(nH=nH))
    G.inject_sources(ijk, ndot)
    G.step(w.dt, 1, 60)
    red = G.reduce()
    lhs = red["photons_initial"] + red["photons_emitted"] + red["photons_floor"]
    rhs = red["photons_stored"] + red["photons_absorbed"] + red["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-4)
    st = G.state_numpy()
    G.step(w.dt, 1)
    out = G.state_numpy()
    G.close()
    g = oracle_grid(st, shape, w.dx, (rt.BC_PERIODIC,) * 6, oracle.CHEM_FULL,
                    sources=(ijk, ndot), clump=LAW_B)
    g.step(w.dt, 1)
    e = errors(out, oracle_state(g))
    print(f"clumped cosmo128 one-step errors {e}", flush=True)
    assert_parity(e, what="clumped cosmo128")
    # the laws act on this run: the unclumped run ends elsewhere
    G0 = rt.RTGrid(rt.make_params(shape, w.dx, prec=rt.PREC_MIXED), dict(nH=nH))
    G0.inject_sources(ijk, ndot)
    G0.step(w.dt, 1, 61)
    x0 = G0.state_numpy()["xHI"]
    G0.close()
    assert float(np.max(np.abs(x0 - out["xHI"]))) > 1e-2
