"""The learned-chemistry step against the FP64 oracle of its own arithmetic
(oracle/surrogate.py), cell by cell, on seeded synthetic states.

Networks with known outputs isolate the step's arithmetic from the network:
with the last layer's weights zero, every cell gets the same predicted
change (exact in both precisions), so the photon accounting (N', F'), the
end state (xHI', T') and the backward-Euler acceptance test are compared
cell by cell against the oracle.  A seeded random network checks the same
with a cell-dependent prediction (the oracle runs the FP64 forward pass on
the bf16-rounded weights and inputs).  Cells whose residual lies within 2%
of the tolerance may be decided either way (the two sides decide in
different precisions); they must then equal one of the two oracle answers.
Features outside the training range must take the exact operator.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from oracle import surrogate as OS
from paper_1004_2503_amd import rt
from paper_1004_2503_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPE = (40, 36, 70)          # nz, ny, nx: ragged tiles in x and y
DX = 3.0e21
TOL = 1e-3
OFF_W4 = sum(o * i + o for o, i in mlp.SIZES[:-1])


def state(seed=4242):
    """Random admissible state; half of the box (z < 20) starts without
    photons, and in a quarter of the box fully neutral too, so that the
    step has dark cells, quiet cells and lit cells."""
    st = W.random_state(SHAPE, seed, nmax=1e-4)
    st["N"][:20] = 0.0
    for k in ("Fx", "Fy", "Fz"):
        st[k][:20] = 0.0
    st["xHI"][:10] = 1.0
    return st


def norm_array(in_min=-60.0, in_max=60.0):
    n = np.concatenate([np.zeros(5), np.ones(5), np.zeros(2), np.ones(2),
                        np.full(5, in_min), np.full(5, in_max)])
    return n.astype(np.float32)


def constant_theta(d_xhi, d_T, seed=1):
    """Network whose output decodes to the changes (d_xhi, d_T) [dex] for
    every cell (zero last-layer weights, bias asinh(d / 1e-3))."""
    th = mlp.init_params(seed)
    th[OFF_W4:OFF_W4 + 128] = 0.0
    th[OFF_W4 + 128:OFF_W4 + 130] = np.arcsinh(np.array([d_xhi, d_T]) / 1e-3)
    return th.astype(np.float32)


def random_theta(seed=7, scale=0.05):
    th = mlp.init_params(seed)
    th[OFF_W4:OFF_W4 + 128] *= scale
    return th.astype(np.float32)


def gpu_step(st, theta, norm, dt, sub_eps, nsub=1, sub=rt.SUB_FIXED, prec=rt.PREC_FP32):
    G = rt.RTGrid(rt.make_params(SHAPE, DX, prec=prec, sub=sub, sub_eps=sub_eps), st)
    th = torch.tensor(theta, device="cuda")
    rt.check(rt.rt_set_surrogate(G.ctx, th, norm, TOL), "rt_set_surrogate")
    G.step(dt, nsub)
    red = G.reduce()
    out = G.state_numpy()
    G.close()
    return out, red


def oracle_step(st, theta, norm, dt, sub_eps, nsub=1, sub=oracle.SUB_FIXED, fp64_thr=0.0):
    p = oracle.make_params(SHAPE, DX, sub=sub, sub_eps=sub_eps)
    return OS.step(p, st, None, dt, nsub, theta.astype(np.float64),
                   norm.astype(np.float64), TOL, select="stiff", fp64_thr=fp64_thr)


def compare(out, red, ref, n_tol=1e-4, rel_net=1e-5):
    """Per-cell comparison; returns (n network cells, n margin cells, n
    fallbacks).  Margin cells (either answer valid): the residual within 2%
    of the tolerance, or the stiffness test within 1e-3 of its threshold."""
    C = rt.C_LIGHT
    Nmax = float(np.abs(ref["N"]).max())
    ex = ref["exact"]
    r = np.maximum(ref["rx"], ref["rT"]) / TOL
    dark = ~(ref["transported"]["N"] > 0)
    margin = (ref["cand"] & (np.abs(r - 1.0) <= 0.02)) | (
        ~dark & (np.abs(ref["stiffness"] - 1.0) <= 1e-3))

    def close(cand):
        eN = np.abs(out["N"] - cand["N"]) / Nmax
        eF = np.maximum.reduce([np.abs(out[k] - cand[k]) for k in ("Fx", "Fy", "Fz")]) / (
            C * Nmax)
        ex_ = np.abs(out["xHI"] - cand["xHI"])
        eT = np.abs(out["T"] - cand["T"]) / cand["T"]
        return (eN <= n_tol) & (eF <= n_tol) & (ex_ <= 1e-3) & (eT <= 1e-3)

    chosen = close({k: ref[k] for k in ("N", "Fx", "Fy", "Fz", "xHI", "T")})
    either = close(ref["net"]) | close(ex)
    # outside the margin: the oracle's choice, to the parity norms
    bad = ~margin & ~chosen
    assert not bad.any(), (
        f"{int(bad.sum())} cells differ; first {np.argwhere(bad)[:5].tolist()}")
    # inside it: either answer
    assert not (margin & ~either).any()
    # accepted cells carry the predicted end state itself
    acc = ref["ok"] & ~margin
    if acc.any():
        assert np.allclose(out["xHI"][acc], ref["net"]["xHI"][acc], rtol=rel_net, atol=0)
        assert np.allclose(out["T"][acc], ref["net"]["T"][acc], rtol=rel_net, atol=0)
    n_fb_oracle = int((ref["cand"] & ~ref["ok"]).sum())
    assert abs(red["n_fallback"] - n_fb_oracle) <= int(margin.sum()), (red["n_fallback"],
                                                                        n_fb_oracle)
    lhs = red["photons_initial"] + red["photons_emitted"] + red["photons_floor"]
    rhs = red["photons_stored"] + red["photons_absorbed"] + red["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-5)
    return int(acc.sum()), int(margin.sum()), n_fb_oracle


# sub_eps = 0 makes every cell that is not dark stiff, so that the network is
# asked everywhere; 0.1 (the adaptive rule's fraction) asks it only where the
# adaptive operator would take more than one sub-cycle
@pytest.mark.parametrize("sub_eps", [0.0, 0.1])
@pytest.mark.parametrize("d", [(0.0, 0.0), (-0.004, 0.002), (-0.3, 0.05)])
def test_constant_prediction_matches_oracle_cell_by_cell(d, sub_eps):
    st = state()
    dt = W.courant_dt(DX)
    theta, norm = constant_theta(*d), norm_array()
    out, red = gpu_step(st, theta, norm, dt, sub_eps)
    ref = oracle_step(st, theta, norm, dt, sub_eps)
    n_acc, n_margin, n_fb = compare(out, red, ref)
    print(f"changes {d}, sub_eps {sub_eps}: {int(ref['cand'].sum())} candidates, {n_acc} "
          f"accepted, {n_fb} fallbacks, {n_margin} at the margin", flush=True)
    if d == (0.0, 0.0) and sub_eps == 0.0:
        assert n_acc > 1000 and n_fb > 1000
    if sub_eps > 0.0:
        assert 1000 < int(ref["cand"].sum()) < int((~(ref["transported"]["N"] <= 0)).sum())


@pytest.mark.parametrize("sub_eps", [0.0, 0.1])
def test_random_network_matches_oracle_cell_by_cell(sub_eps):
    st = state(99)
    dt = W.courant_dt(DX)
    theta, norm = random_theta(), norm_array()
    out, red = gpu_step(st, theta, norm, dt, sub_eps)
    ref = oracle_step(st, theta, norm, dt, sub_eps)
    n_acc, n_margin, n_fb = compare(out, red, ref, n_tol=1e-3, rel_net=2e-4)
    print(f"random network, sub_eps {sub_eps}: {n_acc} accepted, {n_fb} fallbacks, "
          f"{n_margin} at the margin", flush=True)
    if sub_eps == 0.0:
        assert n_acc > 100


def test_mixed_precision_and_adaptive_fallback():
    """Mixed precision: the cells below the FP64 threshold are candidates
    too, and the exact fallback runs adaptively (the oracle's adaptive
    operator)."""
    st = state(5)
    dt = W.courant_dt(DX)
    theta, norm = constant_theta(0.0, 0.0), norm_array()
    out, red = gpu_step(st, theta, norm, dt, 0.1, nsub=16, sub=rt.SUB_ADAPTIVE,
                        prec=rt.PREC_MIXED)
    ref = oracle_step(st, theta, norm, dt, 0.1, nsub=16, sub=oracle.SUB_ADAPTIVE,
                      fp64_thr=1e-3)
    n_acc, n_margin, n_fb = compare(out, red, ref)
    print(f"mixed adaptive: {n_acc} accepted, {n_fb} fallbacks, {n_margin} at the margin, "
          f"{red['n_fp64']} FP64 cells", flush=True)
    assert red["n_fp64"] > 0


def test_out_of_range_features_take_the_exact_operator():
    st = state(7)
    dt = W.courant_dt(DX)
    theta = constant_theta(0.0, 0.0)
    lnh = np.log10(st["nH"].astype(np.float64))
    # in_max of log10 nH near the median, in a gap of the values so that no
    # cell sits where the two precisions could decide differently
    v = np.sort(lnh.ravel())
    j = v.size // 2 + int(np.argmax(np.diff(v[v.size // 2:]) > 1e-4))
    norm = norm_array()
    norm[19] = 0.5 * (v[j] + v[j + 1])
    cut = float(norm[19])
    assert v[j] < cut - 2e-5 and v[j + 1] > cut + 2e-5
    out, red = gpu_step(st, theta, norm, dt, 0.0)
    ref = oracle_step(st, theta, norm, dt, 0.0)
    compare(out, red, ref)
    ood = ref["cand"] & (lnh > cut)
    assert ood.sum() > 1000
    assert not (ref["ok"] & ood).any()
    ex = ref["exact"]
    Nmax = float(np.abs(ex["N"]).max())
    assert np.max(np.abs(out["N"][ood] - ex["N"][ood])) / Nmax <= 1e-4
    assert np.max(np.abs(out["xHI"][ood] - ex["xHI"][ood])) <= 1e-3
    assert red["n_fallback"] >= int(ood.sum())
