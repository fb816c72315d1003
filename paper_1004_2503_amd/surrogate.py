"""Training of the learned chemistry surrogate (not part of the paper's
method; an optional replacement for the exact per-cell operator Phi).

Every numerical step runs in the library: the training pairs -- log10
features, the asinh encoding of the changes and the end values -- from the
exact operator (rt_mlp_pairs), the standardisation (rt_mlp_standardize),
minibatch training with batches drawn on the device, gradient-norm clipping,
the learning-rate schedule and Adam (rt_mlp_train), evaluation, decoding and
the held-out loss (rt_mlp_predict).  This module samples cells, picks pairs
by index and passes arguments.

Features: log10 of nH, xHI, T, N (xHI, N floored at 1e-30) and dt.  The
network predicts u = asinh(d / 1e-3) of the changes d = log10(xHI'/xHI) and
log10(T'/T) over dt.  Most cells move little in one step; a few change by
decades.  Against end values, or against the plain changes, those few set
the standardisation and the quiet majority then carries errors of ~1e-3 in
xHI; the asinh keeps small changes linear and compresses the large ones.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import rt


@dataclass
class Surrogate:
    theta: "object"            # torch float32 (8834,) on the device
    mu_in: np.ndarray
    sd_in: np.ndarray
    mu_out: np.ndarray
    sd_out: np.ndarray
    in_min: np.ndarray
    in_max: np.ndarray
    history: list

    def norm_array(self) -> np.ndarray:
        return np.concatenate([self.mu_in, self.sd_in, self.mu_out, self.sd_out,
                               self.in_min, self.in_max]).astype(np.float32)


def _stream(dev):
    import torch

    return torch.cuda.current_stream(dev).cuda_stream


def _out(like, n, w):
    import torch

    return torch.empty((n, w), dtype=torch.float32, device=like.device)


def features(nH, N, xHI, T, dt):
    """Raw log10 features (n, 5) of cells given as device tensors."""
    n = nH.numel()
    X = _out(nH, n, 5)
    p = rt.make_params((1, 1, 1), 1.0)
    rt.check(rt.rt_mlp_pairs(p, nH, N, xHI, T, dt, 1, X=X, stream=_stream(nH.device)),
             "rt_mlp_pairs")
    return X


def exact_pairs(params, nH, N, xHI, T, dt, nsub, ncycles=None):
    """The exact operator `params` (at most nsub sub-cycles) on copies of the
    given cells (device tensors, dt per cell): returns (X raw features,
    U encoded targets, Y end values log10 xHI', log10 T').  ncycles (device
    int32, optional) receives the sub-cycles each cell took."""
    n = nH.numel()
    X, U, Y = _out(nH, n, 5), _out(nH, n, 2), _out(nH, n, 2)
    rt.check(rt.rt_mlp_pairs(params, nH, N, xHI, T, dt, nsub, X=X, U=U, Yend=Y,
                             ncycles=ncycles, stream=_stream(nH.device)), "rt_mlp_pairs")
    return X, U, Y


def candidate_pairs(params, cells: dict, dt: float, n_keep: int, nsub: int = 64,
                    fp64_thr: float = 0.0, seed: int = 0):
    """Exact pairs weighted towards the cells the step asks the network for.
    The exact adaptive operator `params` (at most nsub sub-cycles) runs on
    every sampled cell; the stiff ones (more than one sub-cycle) and those
    below fp64_thr are all kept, the others fill the rest of n_keep at
    random.  Returns (X, U, Y, number of stiff-or-FP64 pairs kept)."""
    import torch

    n = cells["N"].numel()
    dev = cells["N"].device
    ncyc = torch.zeros(n, dtype=torch.int32, device=dev)
    X, U, Y = exact_pairs(params, cells["nH"], cells["N"], cells["xHI"], cells["T"],
                          torch.full_like(cells["N"], dt), nsub, ncyc)
    hard = (ncyc > 1) | (cells["xHI"] < fp64_thr)
    idx_hard = torch.nonzero(hard).reshape(-1)[:n_keep]
    idx_easy = torch.nonzero(~hard).reshape(-1)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    m = max(0, min(n_keep - idx_hard.numel(), idx_easy.numel()))
    pick = idx_easy[torch.randperm(idx_easy.numel(), generator=g, device=dev)[:m]]
    idx = torch.cat([idx_hard, pick])
    return X[idx], U[idx], Y[idx], int(idx_hard.numel())


def sample_cells(state: dict, n: int, seed: int, lit_fraction: float = 0.8):
    """Draw n cells from a state dict of device tensors (N, xHI, T, nH),
    preferring cells that hold photons (the ones whose chemistry evolves)."""
    import torch

    g = torch.Generator(device=state["N"].device)
    g.manual_seed(seed)
    flatN = state["N"].reshape(-1)
    lit = torch.nonzero(flatN > 0).reshape(-1)
    n_lit = min(int(n * lit_fraction), lit.numel() * 50) if lit.numel() else 0
    idx_lit = lit[torch.randint(0, max(lit.numel(), 1), (n_lit,), generator=g,
                                device=lit.device)] if n_lit else lit[:0]
    idx_any = torch.randint(0, flatN.numel(), (n - n_lit,), generator=g, device=flatN.device)
    idx = torch.cat([idx_lit, idx_any])
    return {k: state[k].reshape(-1)[idx].clone() for k in ("N", "xHI", "T", "nH")}


def perturb_cells(cells: dict, seed: int, frac: float = 0.5, dex_T=(-0.15, 0.25),
                  dex_xhi=(-2.0, 0.3), dex_N=(-0.5, 1.0)):
    """Widen the training inputs beyond the states sampled: a fraction
    `frac` of the cells gets T, xHI and N multiplied by 10^U(lo, hi) dex
    (xHI kept in [1e-12, 1]).  The exact operator labels whatever state it
    is given, so the pairs stay exact; the network then also covers the
    states a run reaches later (hotter ionised gas, lower neutral fractions,
    brighter regions), which its training-range test would otherwise send
    back to the exact operator."""
    import torch

    n = cells["N"].numel()
    g = torch.Generator(device=cells["N"].device)
    g.manual_seed(seed)

    def u(lo, hi):
        return lo + (hi - lo) * torch.rand(n, generator=g, device=cells["N"].device)

    pick = torch.rand(n, generator=g, device=cells["N"].device) < frac
    out = {k: v.clone() for k, v in cells.items()}
    out["T"] = torch.where(pick, cells["T"] * 10.0 ** u(*dex_T), cells["T"])
    out["xHI"] = torch.where(pick, (cells["xHI"] * 10.0 ** u(*dex_xhi)).clamp(1e-12, 1.0),
                             cells["xHI"])
    out["N"] = torch.where(pick, cells["N"] * 10.0 ** u(*dex_N), cells["N"])
    return out


def _init_params(seed: int) -> np.ndarray:
    """He-style uniform initialisation (fan-in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in ((64, 5), (64, 64), (64, 64), (2, 64)):
        lim = math.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def fit(X, U, steps: int = 3000, batch: int = 65536, lr: float = 2e-3, seed: int = 0,
        grad_blocks: int = 256, log_every: int = 250, verbose: bool = True,
        warmup: float = 0.05, clip: float | None = 1.0) -> Surrogate:
    """Fit the network to raw features X (n, 5) and encoded targets U (n, 2),
    device tensors from exact_pairs.  Adam with a learning rate that rises
    linearly over the first `warmup` fraction of the steps and then decays
    as a cosine; the gradient is rescaled to global norm `clip` when above
    it (the changes are heavy tailed: a batch of cells ionised within the
    step can otherwise throw the weights off)."""
    import torch

    dev = X.device
    n = int(X.shape[0])
    rc, h = rt.rt_mlp_create(grad_blocks, _stream(dev))
    rt.check(rc, "rt_mlp_create")
    hist = []
    try:
        st_in = torch.empty(20, dtype=torch.float64, device=dev)
        st_out = torch.empty(8, dtype=torch.float64, device=dev)
        Xs, Us = torch.empty_like(X), torch.empty_like(U)
        rt.check(rt.rt_mlp_standardize(h, X.contiguous(), Xs, st_in), "rt_mlp_standardize")
        rt.check(rt.rt_mlp_standardize(h, U.contiguous(), Us, st_out), "rt_mlp_standardize")
        theta = torch.tensor(_init_params(seed), device=dev)
        m1 = torch.zeros_like(theta)
        m2 = torch.zeros_like(theta)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        opts = rt.rt_mlp_train_opts(batch=min(batch, n), total_steps=steps, lr=lr,
                                    warmup=warmup, lr_floor=1e-5,
                                    clip=0.0 if clip is None else float(clip), beta1=0.9,
                                    beta2=0.999, eps=1e-8, seed=seed)
        t0 = time.time()
        done = 0
        while done < steps:
            k = 1 if done == 0 else min(log_every - done % log_every, steps - done)
            rt.check(rt.rt_mlp_train(h, theta, m1, m2, Xs, Us, opts, done, k, loss),
                     "rt_mlp_train")
            done += k
            lv = float(loss.item())
            hist.append((done, lv, time.time() - t0))
            if verbose:
                print(f"  surrogate step {done}/{steps}: loss {lv:.3e} "
                      f"({time.time() - t0:.1f} s)", flush=True)
        si, so = st_in.cpu().numpy(), st_out.cpu().numpy()
    finally:
        rt.rt_mlp_destroy(h)
    return Surrogate(theta=theta, mu_in=si[0:5], sd_in=si[5:10], mu_out=so[0:2], sd_out=so[2:4],
                     in_min=si[10:15], in_max=si[15:20], history=hist)


def _norm14(s: Surrogate):
    return np.concatenate([s.mu_in, s.sd_in, s.mu_out, s.sd_out]).astype(np.float32)


def mse(s: Surrogate, X, U) -> float:
    """Mean squared standardised error of the network on the pairs (X, U):
    the training loss evaluated on any set of pairs."""
    import torch

    loss = torch.zeros(1, dtype=torch.float64, device=X.device)
    rc, h = rt.rt_mlp_create(1, _stream(X.device))
    rt.check(rc, "rt_mlp_create")
    try:
        rt.check(rt.rt_mlp_predict(h, s.theta, _norm14(s), X.contiguous(), U=U.contiguous(),
                                   loss_dev=loss), "rt_mlp_predict")
        lv = float(loss.item())
    finally:
        rt.rt_mlp_destroy(h)
    return lv


def untrained(s: Surrogate, seed: int = 0) -> Surrogate:
    """The network fit() starts from, with s's standardisation."""
    import torch

    return Surrogate(theta=torch.tensor(_init_params(seed), device=s.theta.device),
                     mu_in=s.mu_in, sd_in=s.sd_in, mu_out=s.mu_out, sd_out=s.sd_out,
                     in_min=s.in_min, in_max=s.in_max, history=[])


def predict(s: Surrogate, X):
    """Raw features -> end values (log10 xHI', log10 T') with the trained
    network (device)."""
    Y = _out(X, int(X.shape[0]), 2)
    rc, h = rt.rt_mlp_create(1, _stream(X.device))
    rt.check(rc, "rt_mlp_create")
    try:
        rt.check(rt.rt_mlp_predict(h, s.theta, _norm14(s), X.contiguous(), Y=Y),
                 "rt_mlp_predict")
    finally:
        rt.rt_mlp_destroy(h)      # waits for the stream
    return Y
