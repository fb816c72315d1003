"""The largest grid the boundary accepts: (nz, ny, nx) = (1597, 1625, 1655),
4,294,931,875 cells = 2^32 - 35,421 (rt_params requires nx ny nz < 2^32),
ragged in all three directions, the library working on caller-owned fields
of 189 GB of HBM.

  * rt_init's FP64 sums of the initial state equal torch's;
  * one mixed-precision step with sources, among them the very last cell:
    sampled 32^3 sub-blocks (the far corner, the last ragged tiles,
    random) equal the oracle stepped from the same inputs, and the photon
    budget closes.

Skipped on a device without the memory for it."""

import numpy as np
import pytest
import torch

import oracle
from paper_1004_2503_amd import rt

from parity_util import assert_parity, errors

pytestmark = pytest.mark.gpu

SHAPE = (1597, 1625, 1655)
DX = 3.0e21
B = 32


def _block(t, o, halo):
    idx = [torch.arange(c - halo, c + B + halo, device=t.device) % n for c, n in zip(o, SHAPE)]
    return t.index_select(0, idx[0]).index_select(1, idx[1]).index_select(2, idx[2]) \
        .double().cpu().numpy()


@pytest.mark.timeout(600)
def test_largest_grid():
    n = int(np.prod(SHAPE))
    assert 2 ** 32 - 262144 < n < 2 ** 32
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 11 * 4 * n + 8 * 2 ** 30:
        pytest.skip(f"needs {11 * 4 * n / 2**30:.0f} GiB of free device memory")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4294)
    mk = lambda: torch.empty(SHAPE, dtype=torch.float32, device="cuda")
    N = [mk(), mk()]
    F = [[mk(), mk()] for _ in range(3)]
    xHI, T, nH = mk(), mk(), mk()
    N[0].uniform_(0.0, 1.0, generator=gen).pow_(3).mul_(1e-3)
    for k in range(3):                       # |F| <= 0.5 c N
        F[k][0].uniform_(-1.0, 1.0, generator=gen).mul_(N[0]).mul_(0.5 * rt.C_LIGHT / 3 ** 0.5)
    xHI.uniform_(-6.0, 0.0, generator=gen).mul_(np.log(10.0)).exp_()
    T.uniform_(2.0, 4.7, generator=gen).mul_(np.log(10.0)).exp_()
    nH.uniform_(-5.0, -1.0, generator=gen).mul_(np.log(10.0)).exp_()
    f = rt.rt_fields()
    f.N[0], f.N[1] = N[0].data_ptr(), N[1].data_ptr()
    f.Fx[0], f.Fx[1] = F[0][0].data_ptr(), F[0][1].data_ptr()
    f.Fy[0], f.Fy[1] = F[1][0].data_ptr(), F[1][1].data_ptr()
    f.Fz[0], f.Fz[1] = F[2][0].data_ptr(), F[2][1].data_ptr()
    f.xHI, f.T, f.nH = xHI.data_ptr(), T.data_ptr(), nH.data_ptr()
    torch.cuda.synchronize()
    params = rt.make_params(SHAPE, DX, prec=rt.PREC_MIXED)
    rc, ctx = rt.rt_init(params, f, None)
    rt.check(rc, "rt_init")
    print("largest grid: initialised", flush=True)
    try:
        rc, red0 = rt.rt_reduce(ctx)
        rt.check(rc, "rt_reduce")
        r0 = red0.as_dict()
        vol = DX ** 3
        assert r0["photons_stored"] == pytest.approx(
            float(N[0].sum(dtype=torch.float64)) * vol, rel=1e-10)
        assert r0["xhi_vol"] == pytest.approx(float(xHI.mean(dtype=torch.float64)), rel=1e-10)
        nz, ny, nx = SHAPE
        ijk = np.array([[nx - 1, ny - 1, nz - 1], [0, 0, 0], [nx - 40, ny - 20, nz - 10],
                        [700, 800, 900]], np.int32)
        ndot = np.array([3e52, 1e51, 2e52, 5e51])
        rt.check(rt.rt_inject_sources(ctx, ijk, ndot), "rt_inject_sources")
        rng = np.random.default_rng(7)
        origins = [(nz - B, ny - B, nx - B), (nz - B, ny - B, 0), (0, ny - B, nx - B),
                   (nz - 20, ny - 40, nx - 60)]
        origins += [tuple(int(rng.integers(0, m - B + 1)) for m in SHAPE) for _ in range(8)]
        before = {o: (_block(xHI, o, 0), _block(T, o, 0)) for o in origins}
        dt = DX / (3 * rt.C_LIGHT)
        rt.check(rt.rt_step(ctx, dt, 2), "rt_step")
        rc, red = rt.rt_reduce(ctx)
        rt.check(rc, "rt_reduce")
        r = red.as_dict()
        print(f"largest grid: stepped, {r['n_fp64']} FP64 cells", flush=True)
        assert r["n_nonfinite"] == 0
        lhs = r["photons_initial"] + r["photons_emitted"] + r["photons_floor"]
        rhs = r["photons_stored"] + r["photons_absorbed"] + r["photons_escaped"]
        assert rhs == pytest.approx(lhs, rel=1e-5)
        rc, cur = rt.rt_current(ctx)
        rt.check(rc, "rt_current")
        p = oracle.make_params((B, B, B), DX, chem=oracle.CHEM_FULL)
        worst = dict(N=0.0, F=0.0, xHI=0.0, T=0.0)
        for o in origins:
            z0, y0, x0 = o
            S = np.zeros((B, B, B))
            for (i, j, k), q in zip(ijk, ndot):
                if z0 <= k < z0 + B and y0 <= j < y0 + B and x0 <= i < x0 + B:
                    S[k - z0, j - y0, i - x0] += q / vol
            res = oracle.step_subblock(p, dt, 2, _block(N[0], o, 1),
                                       [_block(F[k][0], o, 1) for k in range(3)],
                                       before[o][0], before[o][1], _block(nH, o, 0), S)
            ref = dict(N=res[0], Fx=res[1], Fy=res[2], Fz=res[3], xHI=res[4], T=res[5])
            got = dict(N=_block(N[cur], o, 0), Fx=_block(F[0][cur], o, 0),
                       Fy=_block(F[1][cur], o, 0), Fz=_block(F[2][cur], o, 0),
                       xHI=_block(xHI, o, 0), T=_block(T, o, 0))
            e = errors(got, ref)
            for k in worst:
                worst[k] = max(worst[k], e[k])
            assert_parity(e, what=f"largest grid, block at {o}")
        print(f"largest grid: {len(origins)} sampled blocks, worst errors {worst}", flush=True)
    finally:
        rt.lib().rt_destroy(ctx)
        del N, F, xHI, T, nH
        torch.cuda.empty_cache()
