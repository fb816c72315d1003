"""GPU checks of the surrogate's training pipeline in the library (not part
of the paper's method), each against a plain restatement on the host:

  * rt_mlp_pairs: features equal FP64 log10 of the inputs; end values equal
    log10 of rt_chem_apply's results on copies (the same operator), whose
    sub-cycle counts it reproduces bit for bit; targets equal
    asinh(log10(x'/x) / 1e-3) in FP64;
    the inputs are left untouched; features alone skip the chemistry;
  * rt_mlp_standardize: moments against numpy's FP64 mean, std (ddof 1),
    min and max; the same result bit for bit on a rerun;
  * rt_mlp_train: one step equals the explicit step (SplitMix64 indices
    computed here from its published definition, the batch gathered,
    rt_mlp_grad, rt_mlp_adam at the scheduled rate) bit for bit without
    clipping, to float rounding with it; a run split over calls equals one
    call; the schedule's warm-up and cosine phases;
  * rt_mlp_predict: decoded end values and the loss against the same
    network through rt_mlp_forward, destandardised and decoded in FP64."""

import math

import numpy as np
import pytest
import torch

from paper_1004_2503_amd import rt, surrogate

pytestmark = pytest.mark.gpu

DEV = "cuda"
M64 = (1 << 64) - 1


def splitmix64(z):
    z = (z + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def batch_rows(seed, step, batch, n):
    key = splitmix64(seed ^ ((step * 0xD1B54A32D192ED03) & M64))
    return [((splitmix64((key + i) & M64) >> 32) * n) >> 32 for i in range(batch)]


def lr_at(o, s):
    nw = max(int(o.warmup * o.total_steps), 1)
    if s <= nw:
        return o.lr * s / nw
    return o.lr * 0.5 * (1 + math.cos(math.pi * (s - nw) / max(o.total_steps - nw, 1))) + o.lr_floor


def cells(n, seed):
    rng = np.random.default_rng(seed)
    nH = 10 ** rng.uniform(-5, -1, n)
    N = 10 ** rng.uniform(-9, -2, n)
    N[: n // 10] = 0.0
    xHI = 10 ** rng.uniform(-6, 0, n)
    T = 10 ** rng.uniform(1.5, 4.8, n)
    dt = 10 ** rng.uniform(9, 13, n)
    return [torch.tensor(a.astype(np.float32), device=DEV) for a in (nH, N, xHI, T, dt)]


@pytest.mark.parametrize("prec", [rt.PREC_FP32, rt.PREC_MIXED])
def test_pairs_features_targets_and_end_values(prec):
    n = 20011
    nH, N, xHI, T, dt = cells(n, 3)
    keep = [t.clone() for t in (nH, N, xHI, T, dt)]
    p = rt.make_params((1, 1, 1), 1.0, prec=prec, sub=rt.SUB_ADAPTIVE, sub_eps=0.1)
    X = torch.empty((n, 5), device=DEV)
    U = torch.empty((n, 2), device=DEV)
    Y = torch.empty((n, 2), device=DEV)
    nc = torch.zeros(n, dtype=torch.int32, device=DEV)
    rt.check(rt.rt_mlp_pairs(p, nH, N, xHI, T, dt, 64, X, U, Y, nc), "rt_mlp_pairs")
    # the same operator through rt_chem_apply, on copies
    N1, x1, T1 = N.clone(), xHI.clone(), T.clone()
    nc1 = torch.zeros(n, dtype=torch.int32, device=DEV)
    rt.check(rt.rt_chem_apply(p, nH, N1, x1, T1, dt, 64, nc1), "rt_chem_apply")
    torch.cuda.synchronize()
    for a, b in zip((nH, N, xHI, T, dt), keep):
        assert torch.equal(a, b)                 # inputs untouched
    assert torch.equal(nc, nc1)
    f = lambda t: t.cpu().numpy().astype(np.float64)
    ref_X = np.stack([np.log10(f(nH)), np.log10(np.maximum(f(xHI), 1e-30)), np.log10(f(T)),
                      np.log10(np.maximum(f(N), 1e-30)), np.log10(f(dt))], axis=1)
    assert np.allclose(X.cpu().numpy(), ref_X, rtol=2e-7, atol=1e-6)
    lx1 = np.log10(np.maximum(f(x1), 1e-30))
    lt1 = np.log10(f(T1))
    assert np.allclose(Y.cpu().numpy(), np.stack([lx1, lt1], 1), rtol=1e-7, atol=1e-7)
    ref_U = np.stack([np.arcsinh((lx1 - ref_X[:, 1]) / 1e-3),
                      np.arcsinh((lt1 - ref_X[:, 2]) / 1e-3)], axis=1)
    assert np.allclose(U.cpu().numpy(), ref_U, rtol=1e-6, atol=1e-6)
    assert float(U.abs().max()) > 1.0            # some cells change by more than 1e-3 dex
    # features alone
    X2 = surrogate.features(nH, N, xHI, T, dt)
    assert torch.equal(X2, X)


@pytest.mark.parametrize("n,d", [(1_000_003, 5), (77, 2), (1, 3)])
def test_standardize_matches_numpy(n, d):
    rng = np.random.default_rng(n + d)
    A = (rng.standard_normal((n, d)) * rng.uniform(0.1, 10, d) + rng.uniform(-5, 5, d))
    A = A.astype(np.float32)
    At = torch.tensor(A, device=DEV)
    rc, h = rt.rt_mlp_create(1, None)
    rt.check(rc, "rt_mlp_create")
    outs = []
    for _ in range(2):
        out = torch.empty_like(At)
        st = torch.empty(4 * d, dtype=torch.float64, device=DEV)
        rt.check(rt.rt_mlp_standardize(h, At, out, st), "rt_mlp_standardize")
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), st.cpu().numpy()))
    rt.rt_mlp_destroy(h)
    (o1, s1), (o2, s2) = outs
    assert np.array_equal(o1, o2) and np.array_equal(s1.view(np.uint64), s2.view(np.uint64))
    A64 = A.astype(np.float64)
    mu = A64.mean(0)
    sd = np.maximum(A64.std(0, ddof=1), 1e-6) if n > 1 else np.ones(d)
    assert np.allclose(s1[:d], mu, rtol=1e-12, atol=1e-12)
    assert np.allclose(s1[d:2 * d], sd, rtol=1e-10, atol=0.0)
    assert np.array_equal(s1[2 * d:3 * d], A64.min(0)) and np.array_equal(s1[3 * d:], A64.max(0))
    assert np.allclose(o1, ((A64 - mu) / sd).astype(np.float32), rtol=1e-6, atol=1e-6)


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    X = torch.tensor(rng.standard_normal((n, 5)).astype(np.float32), device=DEV)
    Y = torch.tensor(rng.standard_normal((n, 2)).astype(np.float32), device=DEV)
    return X, Y


def _opts(**kw):
    o = dict(batch=1000, total_steps=40, lr=3e-3, warmup=0.1, lr_floor=1e-5, clip=0.0,
             beta1=0.9, beta2=0.999, eps=1e-8, seed=12345)
    o.update(kw)
    return rt.rt_mlp_train_opts(**o)


@pytest.mark.parametrize("clip", [0.0, 0.05])
def test_train_steps_equal_the_explicit_steps(clip):
    n = 50_000
    X, Y = _pairs(n, 1)
    theta0 = torch.tensor(surrogate._init_params(3), device=DEV)
    o = _opts(clip=clip)
    rc, h = rt.rt_mlp_create(64, None)
    rt.check(rc, "rt_mlp_create")
    # library: steps 1-6 (two calls)
    th, m1, m2 = theta0.clone(), torch.zeros_like(theta0), torch.zeros_like(theta0)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    rt.check(rt.rt_mlp_train(h, th, m1, m2, X, Y, o, 0, 2, loss), "rt_mlp_train")
    rt.check(rt.rt_mlp_train(h, th, m1, m2, X, Y, o, 2, 4, loss), "rt_mlp_train")
    # explicit: the same six steps
    te, e1, e2 = theta0.clone(), torch.zeros_like(theta0), torch.zeros_like(theta0)
    g = torch.zeros_like(theta0)
    le = torch.zeros(1, dtype=torch.float64, device=DEV)
    clipped = 0
    for s in range(1, 7):
        idx = torch.tensor(batch_rows(o.seed, s, o.batch, n), device=DEV)
        rt.check(rt.rt_mlp_grad(h, te, X[idx].contiguous(), Y[idx].contiguous(), g, le),
                 "rt_mlp_grad")
        if clip > 0:
            gn = float(torch.sqrt((g.double() ** 2).sum()))
            if gn > clip:
                clipped += 1
            g.mul_(min(1.0, clip / (gn + 1e-12)))
        rt.check(rt.rt_mlp_adam(h, te, e1, e2, g, s, lr_at(o, s)), "rt_mlp_adam")
    torch.cuda.synchronize()
    rt.rt_mlp_destroy(h)
    if clip == 0.0:
        assert torch.equal(th, te) and torch.equal(m1, e1) and torch.equal(m2, e2)
        assert torch.equal(loss, le)
    else:
        assert clipped > 0
        assert torch.allclose(th, te, rtol=1e-5, atol=1e-7)
        assert torch.allclose(m1, e1, rtol=1e-4, atol=1e-9)


def test_schedule_phases_and_split_calls():
    o = _opts(total_steps=100, warmup=0.1)
    assert lr_at(o, 5) == pytest.approx(0.5 * o.lr)
    assert lr_at(o, 100) == pytest.approx(o.lr_floor)
    n = 30_000
    X, Y = _pairs(n, 2)
    rc, h = rt.rt_mlp_create(32, None)
    rt.check(rc, "rt_mlp_create")
    res = []
    for splits in ((0, 100), (0, 1, 37, 100)):
        th = torch.tensor(surrogate._init_params(1), device=DEV)
        m1, m2 = torch.zeros_like(th), torch.zeros_like(th)
        for a, b in zip(splits[:-1], splits[1:]):
            rt.check(rt.rt_mlp_train(h, th, m1, m2, X, Y, o, a, b - a), "rt_mlp_train")
        torch.cuda.synchronize()
        res.append(th.clone())
    assert torch.equal(res[0], res[1])
    th = torch.zeros_like(res[0])
    assert rt.rt_mlp_train(h, th, th, th, X, Y, o, 90, 11) == rt.RT_E_ARG   # past the schedule
    assert rt.rt_mlp_train(h, th, th, th, X, Y, _opts(batch=0), 0, 1) == rt.RT_E_ARG
    rt.rt_mlp_destroy(h)


def test_predict_and_loss_against_forward():
    n = 40_009
    rng = np.random.default_rng(9)
    Xraw = torch.tensor((rng.standard_normal((n, 5)) * 2 - 1).astype(np.float32), device=DEV)
    U = torch.tensor(rng.standard_normal((n, 2)).astype(np.float32), device=DEV)
    theta = torch.tensor(surrogate._init_params(5), device=DEV)
    norm = np.array([0.1, -0.2, 0.3, 0.0, 1.0, 1.5, 2.0, 0.5, 1.0, 3.0, 0.2, -0.1, 1.3, 0.7],
                    np.float32)
    rc, h = rt.rt_mlp_create(1, None)
    rt.check(rc, "rt_mlp_create")
    Y = torch.empty((n, 2), device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    rt.check(rt.rt_mlp_predict(h, theta, norm, Xraw, Y=Y, U=U, loss_dev=loss), "rt_mlp_predict")
    # the same network through rt_mlp_forward on inputs standardised here
    Xs = ((Xraw - torch.tensor(norm[0:5], device=DEV)) / torch.tensor(norm[5:10], device=DEV))
    out = torch.empty((n, 2), device=DEV)
    rt.check(rt.rt_mlp_forward(h, theta, Xs.contiguous(), out), "rt_mlp_forward")
    torch.cuda.synchronize()
    rt.rt_mlp_destroy(h)
    y = out.cpu().numpy().astype(np.float64)
    u = y * norm[12:14] + norm[10:12]
    xr = Xraw.cpu().numpy().astype(np.float64)
    ref = np.stack([xr[:, 1] + 1e-3 * np.sinh(u[:, 0]), xr[:, 2] + 1e-3 * np.sinh(u[:, 1])], 1)
    assert np.allclose(Y.cpu().numpy(), ref, rtol=1e-6, atol=2e-6)
    t = (U.cpu().numpy().astype(np.float64) - norm[10:12]) / norm[12:14]
    ref_loss = float(np.mean((y - t) ** 2))
    assert float(loss.item()) == pytest.approx(ref_loss, rel=1e-5)
