"""The GPU step on the ray-casting problem of the oracle's transport pins (a
point source in a 16^3 box of frozen absorbers, Sec. 2.2): after 400 steps
its steady state equals the oracle's to FP32 rounding, and it meets the same
bounds against brute-force ray casting, with and without a shadowing
clump."""

import numpy as np
import pytest

import oracle
from paper_1004_2503_amd import rt

from test_oracle_raycast import DX, N_CELLS, NDOT, NH0, SRC, check_against_rays, ray_field
from test_oracle_raycast import steady_state as oracle_steady_state

pytestmark = pytest.mark.gpu


def gpu_steady_state(nH, steps=400):
    shp = (N_CELLS,) * 3
    st = dict(N=np.zeros(shp, np.float32), xHI=np.ones(shp, np.float32),
              T=np.full(shp, 1e4, np.float32), nH=nH.astype(np.float32))
    G = rt.RTGrid(rt.make_params(shp, DX, bc=(rt.BC_OUTFLOW,) * 6, chem=rt.CHEM_FROZEN), st)
    G.inject_sources(np.array([SRC], np.int32), np.array([NDOT]))
    G.step(DX / (3 * rt.C_LIGHT), 1, steps)
    red = G.reduce()
    N = G.state_numpy()["N"].astype(np.float64)
    G.close()
    return N, red


@pytest.mark.parametrize("clump", [False, True])
def test_ray_casting_problem(clump):
    nH = np.full((N_CELLS,) * 3, NH0)
    if clump:
        nH[7:10, 7:10, 11:13] *= 50.0
    N, red = gpu_steady_state(nH)
    ref = oracle_steady_state(oracle, nH.astype(np.float32).astype(np.float64))
    err = np.max(np.abs(N - ref)) / np.max(ref)
    print(f"clump={clump}: GPU vs oracle after 400 steps {err:.2e}", flush=True)
    assert err <= 1e-4
    lhs = red["photons_initial"] + red["photons_emitted"] + red["photons_floor"]
    rhs = red["photons_stored"] + red["photons_absorbed"] + red["photons_escaped"]
    assert rhs == pytest.approx(lhs, rel=1e-5)
    if not clump:
        near, mid, every = check_against_rays(N, ray_field(nH, rt.SIGMA_N, rt.C_LIGHT))
        assert 0.75 <= near.min() and near.max() <= 1.35
        assert 0.8 <= mid.min() and mid.max() <= 1.25
        assert abs(np.median(every) - 1.0) < 0.05
    else:
        assert N[8, 8, 14] < 0.2 * N[8, 8, 2]
