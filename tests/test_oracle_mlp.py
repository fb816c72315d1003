"""Pins of the FP64 surrogate-network reference: the hand-written backward
pass against central finite differences (brute force), the bfloat16
rounding helper against its definition on exactly representable and tie
values, and Adam's first step (whose size is lr per coordinate)."""

import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.NPARAM == 8834


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = mlp.init_params(1) + rng.normal(0, 0.05, mlp.NPARAM)
    X = rng.normal(0, 1, (7, 5))
    Y = rng.normal(0, 1, (7, 2))
    _, g = mlp.loss_and_grad(theta, X, Y)
    idx = rng.choice(mlp.NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [0, 319, 320, 383, 384, 8831, 8832, 8833]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        lp, _ = mlp.loss_and_grad(theta + e, X, Y)
        lm, _ = mlp.loss_and_grad(theta - e, X, Y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (k, fd, g[k])


def test_silu_grad_matches_central_differences():
    z = np.linspace(-12, 12, 97)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    assert np.allclose(mlp.silu_grad(z), fd, rtol=1e-7, atol=1e-9)


def test_bf16_round():
    assert mlp.bf16_round(1.0) == 1.0
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0            # tie -> even (down)
    assert mlp.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (up)
    assert mlp.bf16_round(1.0 + 2 ** -7) == 1.0 + 2 ** -7  # representable
    x = np.random.default_rng(0).normal(size=1000)
    r = mlp.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 * (1 + 1e-12))


def test_adam_first_step_has_size_lr():
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 1e-3, -1e3, 0.5])
    new, m, v = mlp.adam_step(theta, np.zeros(5), np.zeros(5), g, 1, lr=1e-3, eps=0.0)
    assert np.allclose(new, -1e-3 * np.sign(g), rtol=1e-12)
