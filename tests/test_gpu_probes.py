"""The bandwidth probes move the data they are timed on: every output of
rt_stream_probe and rt_march_probe is checked bit for bit against the same
FP32 sums in numpy (the kernels add in a fixed order, so the results are
exact), on grids that span several blocks and, for the tile-marching
probe, several 64 x 16 tiles and two 128-plane chunks."""

import numpy as np
import pytest
import torch

from paper_1004_2503_amd import rt

pytestmark = pytest.mark.gpu
DEV = "cuda"


def fsum(vals):
    s = np.zeros_like(vals[0])
    for v in vals:
        s = (s + v).astype(np.float32)
    return s


@pytest.mark.parametrize("nin,nout,n,blocks", [(7, 6, 300_001, 37), (1, 1, 4096, 4),
                                               (16, 16, 65_536, 1024)])
def test_stream_probe_outputs(nin, nout, n, blocks):
    rng = np.random.default_rng(nin * 100 + nout)
    ins_np = [rng.uniform(0.5, 2.0, n).astype(np.float32) for _ in range(nin)]
    ins = [torch.from_numpy(a).to(DEV) for a in ins_np]
    outs = [torch.full((n,), -1.0, dtype=torch.float32, device=DEV) for _ in range(nout)]
    print(f"stream probe nin={nin} nout={nout} n={n} blocks={blocks}", flush=True)
    rc, ms = rt.rt_stream_probe(ins, outs, blocks, 2)
    assert rc == rt.RT_OK and ms > 0.0
    s = fsum(ins_np)
    for k in range(nout):
        v = ins_np[k] if k < nin else np.zeros(n, np.float32)
        assert np.array_equal(outs[k].cpu().numpy(), (s + v).astype(np.float32)), k


def test_march_probe_outputs():
    nz, ny, nx = 256, 48, 192     # 3 x 3 tiles of 64 x 16, two 128-plane chunks
    rng = np.random.default_rng(5)
    ins_np = [rng.uniform(0.5, 2.0, (nz, ny, nx)).astype(np.float32) for _ in range(7)]
    ins = [torch.from_numpy(a).to(DEV) for a in ins_np]
    outs = [torch.full((nz, ny, nx), -1.0, dtype=torch.float32, device=DEV) for _ in range(6)]
    print(f"march probe {nz}x{ny}x{nx}", flush=True)
    rc, ms = rt.rt_march_probe(ins, outs, (nz, ny, nx), 2)
    assert rc == rt.RT_OK and ms > 0.0
    s = fsum(ins_np)
    # each thread adds the plane sum of the thread 64 lanes on, i.e. the
    # next row of its 16-row tile (the last row takes the tile's first)
    y = np.arange(ny)
    partner = (y // 16) * 16 + (y % 16 + 1) % 16
    s2 = (s + s[:, partner, :]).astype(np.float32)
    for k in range(6):
        assert np.array_equal(outs[k].cpu().numpy(), (s2 + ins_np[k]).astype(np.float32)), k


def test_march_probe_rejects_shapes_off_the_tiling():
    ins = [torch.zeros(128 * 16 * 64, dtype=torch.float32, device=DEV) for _ in range(13)]
    for shape in ((128, 16, 32), (64, 16, 64), (128, 8, 64)):
        n = shape[0] * shape[1] * shape[2]
        a = [t[:n] for t in ins]
        rc, _ = rt.rt_march_probe(a[:7], a[7:], shape, 1)
        assert rc == rt.RT_E_ARG, shape
