"""FP64 reference of the learned-chemistry step's own arithmetic.

TEST INFRASTRUCTURE ONLY: the tests use it to check the library's surrogate
form cell by cell; the library never imports it.  Not part of the paper,
which integrates the chemistry exactly: the learned operator is an optional
replacement for the per-cell operator Phi of Appendix A.

A prediction (xHI', T') of the network for a cell holding, after transport,
the photon density N~ and flux F~ (start-of-step xHI, T, density nH, step
dt, clumping factors C_R and C_I of Sec. 3.2.1; x = 1 - xHI) is turned into a
full end state and judged as follows.

Photon accounting.  The photons absorbed are the net ionisations the
prediction implies plus the recombinations and minus the collisional
ionisations over the step, evaluated at the predicted end state:

    P = nH (xHI - xHI') + C_R alpha_B(T') nH^2 x'^2 dt
        - beta(T') nH^2 x' xHI' dt,          clamped to [0, N~],

    N' = N~ - P,   F' = F~ N' / N~,   absorbed += P,

so that the photon budget (emitted = stored + absorbed + escaped) holds
exactly whatever the network predicts.

Acceptance.  The prediction is compared with one backward-Euler step of
length dt of the chemistry of Sec. 2.2 taken with every rate frozen at the
predicted state: the photoionisation rate G' = C_I c sigma_n N', case-B
recombination and collisional ionisation at T' with the electron density
nH x' (Lambda' the cooling of Sec. 2.2's rate set there, the ne nHII terms
times C_R; e_heat the energy per ionisation of the gray constants):

    xHI_BE = (xHI + C_R alpha_B(T') nH x'^2 dt) / (1 + G' dt + beta(T') nH x' dt),
    u_BE = (u0 + P e_heat) / (1 + dt Lambda' / u'),  T_BE = u_BE / (3/2 kB nH (1 + x')),
    u0 = 3/2 kB nH (1 + x) T,   u' = 3/2 kB nH (1 + x') T',

    r_x = |xHI' - xHI_BE|,   r_T = |T' - T_BE| / T'.

Both vanish exactly at the end point of the fully implicit step, and both
measure the prediction's distance from it in the units of the state (an
absolute neutral fraction, a relative temperature).  The cell keeps the prediction when r_x and r_T are at most
the tolerance, its features lie inside the training range, 1e-12 <= xHI' <= 1,
T' >= T_floor and T' is finite; otherwise the exact operator decides it.  Only
the full chemistry (photo-heating and cooling) is ever replaced.

The network itself is the FP64 forward pass of ``oracle.mlp`` on the
standardised log10 features (nH, xHI, T, N~, dt; xHI and N~ floored at
1e-30); its two outputs, de-standardised, are u = asinh(d / 1e-3) of the
changes d of log10 xHI and log10 T over the step.
"""

from __future__ import annotations

import numpy as np

from . import (CHEM_FULL, CHEM_OFF, Grid, Params, chem_timescale, clumping,
               heat_per_ionisation_erg, mlp, rates_n)

FLOOR = 1e-30
DSCALE = 1e-3
XHI_MIN = 1e-12
KB = 1.380649e-16


def features(nH, N, xHI, T, dt) -> np.ndarray:
    """(n, 5) log10 features: nH, max(xHI, 1e-30), T, max(N, 1e-30), dt."""
    nH, N, xHI, T = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (nH, N, xHI, T))
    dt = np.broadcast_to(np.asarray(dt, dtype=np.float64), nH.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.stack([np.log10(nH), np.log10(np.maximum(xHI, FLOOR)), np.log10(T),
                         np.log10(np.maximum(N, FLOOR)), np.log10(dt)], axis=1)


def split_norm(norm):
    """The 24 standardisation values: mu_in, sd_in, mu_out, sd_out, in_min, in_max."""
    n = np.asarray(norm, dtype=np.float64).reshape(-1)
    assert n.size == 24
    return dict(mu_in=n[0:5], sd_in=n[5:10], mu_out=n[10:12], sd_out=n[12:14],
                in_min=n[14:19], in_max=n[19:24])


def out_of_range(f, norm) -> np.ndarray:
    """True where a feature leaves the training range (or is not a number)."""
    s = split_norm(norm)
    inside = (f >= s["in_min"]) & (f <= s["in_max"])
    return ~inside.all(axis=1)


def network_outputs(theta, norm, f, bf16_operands: bool = True) -> np.ndarray:
    """Standardised network outputs (n, 2) for features f.  With
    bf16_operands the weights and the standardised inputs are first rounded
    to bfloat16, the operand precision of the matrix-core kernels (biases
    stay as given); the arithmetic is FP64 either way."""
    s = split_norm(norm)
    x = (np.asarray(f, dtype=np.float64) - s["mu_in"]) / s["sd_in"]
    th = np.asarray(theta, dtype=np.float64).copy()
    if bf16_operands:
        x = mlp.bf16_round(x)
        off = 0
        for o, i in mlp.SIZES:
            th[off:off + o * i] = mlp.bf16_round(th[off:off + o * i])
            off += o * i + o
    y, _ = mlp.forward(th, x)
    return y


def decode(f, y, norm):
    """Standardised outputs -> predicted end values (xHI', T')."""
    s = split_norm(norm)
    u = np.asarray(y, dtype=np.float64) * s["sd_out"] + s["mu_out"]
    d = DSCALE * np.sinh(u)
    return 10.0 ** (f[:, 1] + d[:, 0]), 10.0 ** (f[:, 2] + d[:, 1])


def accounting(params: Params, dt, nH, Nt, Fx, Fy, Fz, xHI, T, xs, Ts, tol, ood,
               rates=rates_n, clump=clumping):
    """Photon accounting and acceptance test of predictions (xs, Ts) for
    cells (arrays of one length).  ``rates(T) -> (n, 6)`` and
    ``clump(params, nH) -> (C_R, C_I)`` are the oracle's own unless a test
    substitutes them.  Returns a dict of arrays: P, N, Fx, Fy, Fz, xHI, T
    (the end state if accepted), rx, rT and ok."""
    a = [np.asarray(v, dtype=np.float64).reshape(-1) for v in
         (nH, Nt, Fx, Fy, Fz, xHI, T, xs, Ts)]
    nH, Nt, Fx, Fy, Fz, xHI, T, xs, Ts = a
    n = nH.size
    CR = np.empty(n)
    CI = np.empty(n)
    for i in range(n):
        CR[i], CI[i] = clump(params, nH[i])
    r = rates(np.where(np.isfinite(Ts) & (Ts > 0), Ts, 1.0))
    alpha, beta = r[:, 0], r[:, 1]
    x0 = 1.0 - xHI
    x1 = 1.0 - xs
    # photons absorbed: net ionisations + recombinations - collisional
    # ionisations at the predicted end state
    P = (nH * (xHI - xs) + CR * alpha * nH * nH * x1 * x1 * dt -
         beta * nH * nH * x1 * xs * dt)
    P = np.minimum(np.maximum(P, 0.0), Nt)
    Ns = Nt - P
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(Nt > 0.0, Ns / Nt, 0.0)
    csig = params.c * params.sigma_n
    # neutral fraction after one backward-Euler step with the rates frozen
    # at the prediction
    xBE = (xHI + CR * alpha * nH * x1 * x1 * dt) / (1.0 + CI * csig * Ns * dt +
                                                     beta * nH * x1 * dt)
    rx = np.abs(xs - xBE)
    # energy: backward Euler with the cooling rate at the predicted state
    lam = nH * nH * (CR * x1 * x1 * (r[:, 2] + r[:, 5]) + x1 * xs * (r[:, 3] + r[:, 4]))
    u0 = 1.5 * KB * nH * (1.0 + x0) * T
    us = 1.5 * KB * nH * (1.0 + x1) * Ts
    with np.errstate(divide="ignore", invalid="ignore"):
        uBE = (u0 + P * heat_per_ionisation_erg(params)) / (1.0 + dt * lam / us)
        TBE = uBE / (1.5 * KB * nH * (1.0 + x1))
        rT = np.abs(Ts - TBE) / Ts
    full = params.chem == CHEM_FULL
    ok = (full & ~np.asarray(ood, dtype=bool) & (xs >= XHI_MIN) & (xs <= 1.0) &
          (Ts >= params.T_floor) & np.isfinite(Ts) & (rx <= tol) & (rT <= tol))
    return dict(P=P, N=Ns, Fx=Fx * scale, Fy=Fy * scale, Fz=Fz * scale, xHI=xs, T=Ts,
                rx=rx, rT=rT, ok=ok)


def stiffness(params: Params, dt, nH, N, xHI, T) -> np.ndarray:
    """sub_eps times the chemistry time scale over the step, per cell (at the
    transported state): below 1 the adaptive operator would take more than
    one sub-cycle (the cell is stiff)."""
    nH, N, xHI, T = (np.asarray(v, dtype=np.float64).reshape(-1) for v in (nH, N, xHI, T))
    out = np.empty(nH.size)
    for i in range(nH.size):
        out[i] = params.sub_eps * chem_timescale(params, nH[i], N[i], xHI[i], T[i]) / dt
    return out


def _clone(params: Params, **kw) -> Params:
    q = Params.from_buffer_copy(params)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def step(params: Params, state: dict, sources, dt, nsub, theta, norm, tol,
         select: str = "stiff", fp64_thr: float = 0.0, bf16_operands: bool = True) -> dict:
    """One step of the learned form on a grid.  Transport (the oracle's step
    with chemistry off), then per cell: dark, fully neutral cells (no
    photons after transport, xHI = 1) take the exact operator (the oracle's
    step with the chemistry of `params`), and so, with select = "stiff", do
    the cells that the adaptive operator would finish in one sub-cycle,
    unless their xHI lies below fp64_thr (the mixed form sends those cells to
    the network too); the other cells (the candidates; with select = "lit"
    every cell that is not dark) take the network's prediction where it is
    accepted and the exact operator elsewhere.  Returns the end state (N,
    Fx, Fy, Fz, xHI, T) plus per-cell arrays cand, ok, rx, rT, P, stiffness
    (see stiffness()), the exact end state ("exact"), the transported state
    ("transported") and the end state every cell would have if its
    prediction were accepted ("net")."""
    shape = np.shape(state["nH"])

    def run(p, nsub_):
        g = Grid(p)
        g.set_state(**{k: np.asarray(state[k], dtype=np.float64) for k in
                       ("N", "Fx", "Fy", "Fz", "xHI", "T", "nH")})
        if sources is not None:
            g.set_sources(*sources)
        g.step(dt, nsub_)
        return dict(N=g.N.copy(), Fx=g.Fx.copy(), Fy=g.Fy.copy(), Fz=g.Fz.copy(),
                    xHI=g.xHI.copy(), T=g.T.copy(), tally=g.tally.copy())

    tr = run(_clone(params, chem=CHEM_OFF), 1)
    ex = run(params, nsub)
    nH = np.asarray(state["nH"], dtype=np.float64).reshape(-1)
    x0 = np.asarray(state["xHI"], dtype=np.float64).reshape(-1)
    T0 = np.asarray(state["T"], dtype=np.float64).reshape(-1)
    Nt = tr["N"].reshape(-1)
    dark = ~(Nt > 0.0) & (x0 >= 1.0)
    cand = ~dark
    ratio = stiffness(params, dt, nH, Nt, x0, T0)
    if select == "stiff":
        cand &= (ratio < 1.0) | (x0 < fp64_thr)
    elif select != "lit":
        raise ValueError(select)
    f = features(nH, Nt, x0, T0, dt)
    y = network_outputs(theta, norm, f, bf16_operands)
    xs, Ts = decode(f, y, norm)
    acc = accounting(params, dt, nH, Nt, tr["Fx"].reshape(-1), tr["Fy"].reshape(-1),
                     tr["Fz"].reshape(-1), x0, T0, xs, Ts, tol, out_of_range(f, norm))
    ok = cand & acc["ok"]
    out = {}
    for k in ("N", "Fx", "Fy", "Fz", "xHI", "T"):
        out[k] = np.where(ok, acc[k], ex[k].reshape(-1)).reshape(shape)
    out.update(cand=cand.reshape(shape), ok=ok.reshape(shape), rx=acc["rx"].reshape(shape),
               stiffness=ratio.reshape(shape),
               rT=acc["rT"].reshape(shape), P=acc["P"].reshape(shape), exact=ex,
               transported=tr,
               net={k: acc[k].reshape(shape) for k in ("N", "Fx", "Fy", "Fz", "xHI", "T")})
    return out
