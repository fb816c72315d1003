"""Helpers shared by the GPU parity tests: run the library and the FP64
oracle on the same FP32-representable inputs and measure their difference
with the per-field norms used throughout the tests:

  N    max |dN| / max |N_oracle|
  F    max_k max |dF_k| / (c max |N_oracle|)
  xHI  max |dxHI|                  (absolute: xHI lies in [0, 1])
  T    max |dT| / T_oracle          (pointwise relative)
"""

from __future__ import annotations

import numpy as np

import oracle
from paper_1004_2503_amd import rt

C = rt.C_LIGHT
TOL = dict(N=1e-4, F=1e-4, xHI=1e-3, T=1e-3)
FIELDS = ("N", "Fx", "Fy", "Fz", "xHI", "T")


def gpu_params(shape, dx, bc, chem, prec=rt.PREC_FP32, sub=rt.SUB_FIXED, sub_eps=0.1,
               clump=None, flux=rt.FLUX_LF):
    return rt.make_params(shape, dx, bc=bc, chem=chem, prec=prec, sub=sub, sub_eps=sub_eps,
                          clump=clump, flux=flux)


def oracle_grid(state, shape, dx, bc, chem, sub=oracle.SUB_FIXED, sub_eps=0.1, sources=None,
                clump=None, flux=oracle.FLUX_LF, hubble=0.0):
    p = oracle.make_params(shape, dx, bc=bc, chem=chem, sub=sub, sub_eps=sub_eps, clump=clump,
                           flux=flux, hubble=hubble)
    g = oracle.Grid(p)
    g.set_state(**{k: np.asarray(state[k], dtype=np.float64) for k in
                   ("N", "Fx", "Fy", "Fz", "xHI", "T", "nH") if k in state})
    if sources is not None:
        g.set_sources(*sources)
    return g


def errors(gpu: dict, ref: dict) -> dict:
    Nmax = float(np.max(np.abs(ref["N"]))) or 1.0
    e = {}
    e["N"] = float(np.max(np.abs(gpu["N"] - ref["N"]))) / Nmax
    e["F"] = max(float(np.max(np.abs(gpu[k] - ref[k]))) for k in ("Fx", "Fy", "Fz")) / (C * Nmax)
    e["xHI"] = float(np.max(np.abs(gpu["xHI"] - ref["xHI"])))
    e["T"] = float(np.max(np.abs(gpu["T"] - ref["T"]) / ref["T"]))
    return e


def assert_parity(e: dict, tol: dict = TOL, what: str = ""):
    bad = {k: (e[k], tol[k]) for k in tol if not e[k] <= tol[k]}
    assert not bad, f"{what}: parity failed {bad} (all errors {e})"


def oracle_state(g) -> dict:
    return dict(N=g.N.copy(), Fx=g.Fx.copy(), Fy=g.Fy.copy(), Fz=g.Fz.copy(),
                xHI=g.xHI.copy(), T=g.T.copy())


def one_step_pair(state, shape, dx, dt, nsub, bc, chem, prec=rt.PREC_FP32,
                  sub=rt.SUB_FIXED, sub_eps=0.1, sources=None, clump=None, flux=rt.FLUX_LF,
                  hubble=0.0, nsteps=1):
    """Step the library and the oracle from the same state (``clump``: None
    or the (cr_norm, cr_exp, ci_norm, ci_exp) laws on both sides; ``flux``
    the intercell flux, LF or HLL, the same code on both sides; ``hubble``
    the expansion rate H; ``nsteps`` steps on both sides).
    Returns (gpu numpy state, oracle numpy state, gpu reductions, oracle grid)."""
    G = rt.RTGrid(gpu_params(shape, dx, bc, chem, prec, sub, sub_eps, clump, flux), state)
    if sources is not None:
        G.inject_sources(*sources)
    if hubble:
        G.set_expansion(hubble)
    G.step(dt, nsub, nsteps)
    red = G.reduce(allow_nonfinite=True)
    out = G.state_numpy()
    G.close()
    g = oracle_grid(state, shape, dx, bc, chem, sub, sub_eps, sources, clump, flux, hubble)
    g.step(dt, nsub, nsteps)
    return out, oracle_state(g), red, g
