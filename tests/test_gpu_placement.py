"""The binding's field placement (one allocation, field k starting k * 256
bytes past a 256-byte-aligned stride) changes where the streams land in HBM,
never the arithmetic: a grid so laid out and one on separately allocated
fields give bit-identical states and sums after several steps (LF and HLL,
sources, deferred FP64 cells)."""

import numpy as np
import pytest
import torch

from paper_1004_2503_amd import rt
from paper_1004_2503_amd import workloads as W

pytestmark = pytest.mark.gpu

DX = 3.0e21
DT = W.courant_dt(DX)


def separate_context(params, st, shape, ijk, ndot):
    dev = torch.device("cuda")
    t = {}
    for name in ("N", "Fx", "Fy", "Fz"):
        t[name] = [torch.as_tensor(st[name]).to(dev).reshape(shape).contiguous().clone(),
                   torch.zeros(shape, dtype=torch.float32, device=dev)]
    for name in ("xHI", "T", "nH"):
        t[name] = torch.as_tensor(st[name]).to(dev).reshape(shape).contiguous().clone()
    f = rt.rt_fields()
    for name in ("N", "Fx", "Fy", "Fz"):
        getattr(f, name)[0] = t[name][0].data_ptr()
        getattr(f, name)[1] = t[name][1].data_ptr()
    f.xHI, f.T, f.nH = t["xHI"].data_ptr(), t["T"].data_ptr(), t["nH"].data_ptr()
    torch.cuda.synchronize()
    rc, ctx = rt.rt_init(params, f, torch.cuda.current_stream().cuda_stream)
    rt.check(rc, "rt_init")
    rt.check(rt.rt_inject_sources(ctx, ijk, ndot), "rt_inject_sources")
    return ctx, t


@pytest.mark.parametrize("flux", [rt.FLUX_LF, rt.FLUX_HLL])
def test_staggered_layout_is_bit_identical_to_separate_fields(flux):
    shape = (26, 37, 130)
    st = W.random_state(shape, seed=900 + flux)
    st = {k: np.asarray(v, dtype=np.float32) for k, v in st.items()}
    for k in ("N", "Fx", "Fy", "Fz"):
        st.setdefault(k, np.zeros(shape, np.float32))
    rng = np.random.default_rng(4)
    ijk = np.stack([rng.integers(0, shape[2], 30), rng.integers(0, shape[1], 30),
                    rng.integers(0, shape[0], 30)], axis=1).astype(np.int32)
    ndot = 10 ** rng.uniform(50, 53, 30)
    params = rt.make_params(shape, DX, prec=rt.PREC_MIXED, flux=flux, sub=rt.SUB_ADAPTIVE,
                            sub_eps=0.1)
    print(f"placement: flux={flux} shape={shape}", flush=True)
    G = rt.RTGrid(params, st)
    # the documented layout: views of one allocation at the staggered stride
    ncell = shape[0] * shape[1] * shape[2]
    stride = (ncell + 63) // 64 * 64 + rt.FIELD_STAGGER
    base = G.N[0].data_ptr()
    ptrs = [G.N[0], G.N[1], G.Fx[0], G.Fx[1], G.Fy[0], G.Fy[1], G.Fz[0], G.Fz[1], G.xHI, G.T,
            G.nH]
    assert [p.data_ptr() - base for p in ptrs] == [4 * k * stride for k in range(11)]
    assert base % 256 == 0
    G.inject_sources(ijk, ndot)
    G.step(DT, 1, 4)
    out_a, red_a = G.state_numpy(), G.reduce()
    G.close()

    ctx, keep = separate_context(params, st, shape, ijk, ndot)
    for _ in range(4):
        rt.check(rt.rt_step(ctx, DT, 1), "rt_step")
    rc, red_b = rt.rt_reduce(ctx)
    rt.check(rc, "rt_reduce")
    red_b = red_b.as_dict()
    out_b = {}
    for name, fid in (("N", rt.FIELD_N), ("Fx", rt.FIELD_FX), ("Fy", rt.FIELD_FY),
                      ("Fz", rt.FIELD_FZ), ("xHI", rt.FIELD_XHI), ("T", rt.FIELD_T)):
        a = np.empty(shape, np.float32)
        rt.check(rt.rt_state(ctx, fid, a.ctypes.data, False), "rt_state")
        out_b[name] = a
    rt.rt_destroy(ctx)
    del keep
    for k in out_b:
        assert np.array_equal(out_a[k].view(np.uint32), out_b[k].view(np.uint32)), k
    for k in ("xhi_vol", "photons_stored", "photons_absorbed", "n_fp64"):
        assert red_a[k] == red_b[k], k
    assert red_a["n_fp64"] > 0
