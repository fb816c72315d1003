"""The allocation-free network gradient rt_mlp_grad_noalloc against the
workspace form rt_mlp_grad, through the C ABI: two calls in a row, the
second on a smaller batch with fewer gradient blocks, each equal bit for bit
to rt_mlp_grad with the same number of blocks (the same kernels and
summation order); then the size limit of the fixed scratch."""

import pytest
import torch

from paper_1004_2503_amd import rt

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _data(B, seed):
    g = torch.Generator(device=DEV).manual_seed(seed)
    theta = 0.2 * torch.randn(rt.MLP_NPARAM, generator=g, device=DEV)
    X = torch.randn(B, 5, generator=g, device=DEV)
    Y = torch.randn(B, 2, generator=g, device=DEV)
    return theta, X, Y


def _workspace_grad(blocks, theta, X, Y):
    rc, m = rt.rt_mlp_create(blocks)
    rt.check(rc, "rt_mlp_create")
    g = torch.empty(rt.MLP_NPARAM, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    rt.check(rt.rt_mlp_grad(m, theta, X, Y, g, loss), "rt_mlp_grad")
    torch.cuda.synchronize()
    rt.check(rt.rt_mlp_destroy(m), "rt_mlp_destroy")
    return g, loss


def test_noalloc_grad_equals_workspace_grad_on_two_calls():
    torch.cuda.set_device(0)
    for blocks, B, seed in ((rt.MLP_NOALLOC_BLOCKS, 100_003, 1), (37, 4_099, 2)):
        theta, X, Y = _data(B, seed)
        g = torch.full((rt.MLP_NPARAM,), float("nan"), device=DEV)
        loss = torch.zeros(1, dtype=torch.float64, device=DEV)
        rt.check(rt.rt_mlp_grad_noalloc(blocks, theta, X, Y, g, loss), "rt_mlp_grad_noalloc")
        torch.cuda.synchronize()
        gw, lw = _workspace_grad(blocks, theta, X, Y)
        assert bool(torch.isfinite(g).all()) and float(g.abs().max()) > 0.0
        assert torch.equal(g, gw), float((g - gw).abs().max())
        assert torch.equal(loss, lw)


def test_noalloc_grad_rejects_sizes_beyond_its_scratch():
    theta, X, Y = _data(64, 3)
    g = torch.empty(rt.MLP_NPARAM, device=DEV)
    assert rt.rt_mlp_grad_noalloc(rt.MLP_NOALLOC_BLOCKS + 1, theta, X, Y, g) == rt.RT_E_SCRATCH
    assert rt.rt_mlp_grad_noalloc(0, theta, X, Y, g) == rt.RT_E_ARG
