"""Training of the learned chemistry surrogate (not part of the paper's
method; an optional replacement for the exact per-cell operator Phi).

Everything numerical runs in the library: training pairs come from the exact
operator on the GPU (rt_chem_apply), gradients and Adam steps from the
matrix-core kernels (rt_mlp_grad, rt_mlp_adam), evaluation from
rt_mlp_forward.  This module only samples cells, builds the log-space
features, standardises them and loops.

Features (log10, floored at 1e-30 for N and xHI): nH, xHI, T, N, dt.
The network predicts u = asinh(d / DSCALE) of the changes d = log10(xHI'/xHI)
and log10(T'/T) over dt.  Most cells move little in one step; a few change
by decades.  Against end values, or against the plain changes, those few set
the standardisation and the quiet majority then carries errors of ~1e-3 in
xHI; the asinh keeps small changes linear and compresses the large ones.
fit() and predict() take and return the end values log10 xHI', log10 T';
the conversion happens inside.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import rt

FLOOR = 1e-30
DSCALE = 1e-3     # [dex]: changes below it are learnt linearly


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


def features(torch, nH, N, xHI, T, dt):
    return torch.stack([torch.log10(nH), torch.log10(xHI.clamp_min(FLOOR)), torch.log10(T),
                        torch.log10(N.clamp_min(FLOOR)), torch.log10(dt)], dim=1)


def exact_pairs(params, nH, N, xHI, T, dt, nsub, ncycles=None):
    """Apply the exact operator to copies of the given cells (device tensors);
    returns (X raw features, Y raw targets, N after).  ncycles (device
    int32, optional) receives the sub-cycles each cell took."""
    import torch

    N1, x1, T1 = N.clone(), xHI.clone(), T.clone()
    rt.check(rt.rt_chem_apply(params, nH, N1, x1, T1, dt, nsub, ncycles), "rt_chem_apply")
    X = features(torch, nH, N, xHI, T, dt)
    Y = torch.stack([torch.log10(x1.clamp_min(FLOOR)), torch.log10(T1)], dim=1)
    return X, Y, N1


def candidate_pairs(params, cells: dict, dt: float, n_keep: int, nsub: int = 64,
                    fp64_thr: float = 0.0, seed: int = 0):
    """Exact pairs weighted towards the cells the step asks the network for.
    The exact adaptive operator `params` (at most nsub sub-cycles) runs on
    every sampled cell; the stiff ones (more than one sub-cycle) and those
    below fp64_thr are all kept, the others fill the rest of n_keep at
    random.  Returns (X, Y, number of stiff-or-FP64 pairs kept)."""
    import torch

    n = cells["N"].numel()
    dev = cells["N"].device
    ncyc = torch.zeros(n, dtype=torch.int32, device=dev)
    X, Y, _ = exact_pairs(params, cells["nH"], cells["N"], cells["xHI"], cells["T"],
                          torch.full_like(cells["N"], dt), nsub, ncyc)
    hard = (ncyc > 1) | (cells["xHI"] < fp64_thr)
    idx_hard = torch.nonzero(hard).reshape(-1)[:n_keep]
    idx_easy = torch.nonzero(~hard).reshape(-1)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    m = max(0, min(n_keep - idx_hard.numel(), idx_easy.numel()))
    pick = idx_easy[torch.randperm(idx_easy.numel(), generator=g, device=dev)[:m]]
    idx = torch.cat([idx_hard, pick])
    return X[idx], Y[idx], int(idx_hard.numel())


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


def fit(X, Y, steps: int = 3000, batch: int = 65536, lr: float = 2e-3, seed: int = 0,
        grad_blocks: int = 512, log_every: int = 250, verbose: bool = True,
        warmup: float = 0.05, clip: float | None = 1.0) -> Surrogate:
    """Fit the network to raw features X (n, 5) and end values Y (n, 2) =
    (log10 xHI', log10 T'), device tensors; it learns encode(X, Y).  Adam
    with a learning rate that rises linearly over the first
    `warmup` fraction of the steps and then decays as a cosine; the gradient
    is rescaled to global norm `clip` when above it (the changes are heavy
    tailed: a batch of cells ionised within the step can otherwise throw the
    weights off)."""
    import torch

    dev = X.device
    Y = encode(X, Y)                        # end values -> asinh of changes
    mu_in, sd_in = X.mean(0), X.std(0).clamp_min(1e-6)
    mu_out, sd_out = Y.mean(0), Y.std(0).clamp_min(1e-6)
    Xs = ((X - mu_in) / sd_in).float().contiguous()
    Ys = ((Y - mu_out) / sd_out).float().contiguous()
    n = Xs.shape[0]
    theta = torch.tensor(_init_params(seed), device=dev)
    m1 = torch.zeros_like(theta)
    m2 = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    rc, h = rt.rt_mlp_create(grad_blocks, torch.cuda.current_stream(dev).cuda_stream)
    rt.check(rc, "rt_mlp_create")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    hist = []
    t0 = time.time()
    try:
        for step in range(1, steps + 1):
            idx = torch.randint(0, n, (min(batch, n),), generator=g, device=dev)
            xb, yb = Xs[idx].contiguous(), Ys[idx].contiguous()
            rt.check(rt.rt_mlp_grad(h, theta, xb, yb, grad, loss), "rt_mlp_grad")
            if clip is not None:
                gn = torch.linalg.vector_norm(grad)
                grad.mul_(torch.clamp(clip / (gn + 1e-12), max=1.0))
            nw = max(int(warmup * steps), 1)
            if step <= nw:
                lr_t = lr * step / nw
            else:
                lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - nw) / max(steps - nw, 1))) + 1e-5
            rt.check(rt.rt_mlp_adam(h, theta, m1, m2, grad, step, lr_t), "rt_mlp_adam")
            if step == 1 or step % log_every == 0 or step == steps:
                lv = float(loss.item())
                hist.append((step, lv, time.time() - t0))
                if verbose:
                    print(f"  surrogate step {step}/{steps}: loss {lv:.3e} "
                          f"({time.time() - t0:.1f} s)", flush=True)
    finally:
        rt.rt_mlp_destroy(h)
    return Surrogate(theta=theta, mu_in=mu_in.cpu().numpy(), sd_in=sd_in.cpu().numpy(),
                     mu_out=mu_out.cpu().numpy(), sd_out=sd_out.cpu().numpy(),
                     in_min=X.min(0).values.cpu().numpy(), in_max=X.max(0).values.cpu().numpy(),
                     history=hist)


def encode(X, Y):
    """End values Y = (log10 xHI', log10 T') -> network targets
    asinh((Y - (log10 xHI, log10 T)) / DSCALE)."""
    import torch

    return torch.asinh((Y - X[:, 1:3]) / DSCALE)


def decode(X, U):
    """Network outputs (destandardised) -> end values."""
    import torch

    return X[:, 1:3].float() + DSCALE * torch.sinh(U)


def mse(s: Surrogate, X, Y) -> float:
    """Mean squared standardised error of the network on (X, end values Y):
    the training loss evaluated on any set of pairs."""
    import torch

    U = _outputs(s, X)
    so = torch.tensor(s.sd_out, device=X.device)
    return float((((U - encode(X, Y).float()) / so) ** 2).mean())


def untrained(s: Surrogate, seed: int = 0) -> Surrogate:
    """The network fit() starts from, with s's standardisation."""
    import torch

    return Surrogate(theta=torch.tensor(_init_params(seed), device=s.theta.device),
                     mu_in=s.mu_in, sd_in=s.sd_in, mu_out=s.mu_out, sd_out=s.sd_out,
                     in_min=s.in_min, in_max=s.in_max, history=[])


def predict(s: Surrogate, X):
    """Raw features -> end values (log10 xHI', log10 T') with the trained
    network (device)."""
    return decode(X, _outputs(s, X))


def _outputs(s: Surrogate, X):
    """Raw features -> destandardised network outputs (asinh of changes)."""
    import torch

    Xs = ((X - torch.tensor(s.mu_in, device=X.device)) /
          torch.tensor(s.sd_in, device=X.device)).float().contiguous()
    Y = torch.zeros((X.shape[0], 2), device=X.device)
    rc, h = rt.rt_mlp_create(1, torch.cuda.current_stream(X.device).cuda_stream)
    rt.check(rc, "rt_mlp_create")
    try:
        rt.check(rt.rt_mlp_forward(h, s.theta, Xs, Y), "rt_mlp_forward")
    finally:
        torch.cuda.synchronize()
        rt.rt_mlp_destroy(h)
    return Y * torch.tensor(s.sd_out, device=X.device) + torch.tensor(s.mu_out, device=X.device)
