"""Transport physics of the oracle against brute-force ray casting (method
error, not parity): a point source in a 16^3 box of frozen absorbers
(chemistry off, absorption on: Sec. 2.2 kappa = sigma_n n_HI) run to its
steady state, against

    N_ray(r) = Ndot exp(-tau) / (4 pi r^2 c),

tau the optical depth from the source to each cell centre by exact cell
traversal (every crossing of a grid plane along the segment; the
cell-centred opacity times the length inside each cell).

  * the traversal itself: uniform opacity gives kappa r exactly; a diagonal
    through a single opaque cell picks up its whole diagonal chord;
  * uniform medium: the M1 steady state agrees with the ray answer within
    25% beyond 4 cells and 35% between 3 and 4 (the closure and the
    first-order fluxes spread the beam; the median over the box is within
    5%);
  * a dense clump casts a shadow (Sec. 2.2: the M1 closure keeps the
    directionality that lets an opaque region shade what lies behind it):
    behind it N drops to a fraction of its mirror image, while cells off the
    shadow keep the uniform-medium solution."""

import numpy as np
import pytest

N_CELLS = 16
DX = 3.4e20
NH0 = 1e-4           # kappa dx = 0.1 with xHI = 1
SRC = (8, 8, 8)
NDOT = 1e50


def siddon_tau(src, dst, kappa, dx):
    """Optical depth along the segment between the centres of cells src and
    dst ((i, j, k) = (x, y, z)); kappa is (nz, ny, nx) [1/cm]."""
    p0 = np.asarray(src, float) + 0.5
    p1 = np.asarray(dst, float) + 0.5
    d = p1 - p0
    ts = [0.0, 1.0]
    for ax in range(3):
        if d[ax] != 0.0:
            lo, hi = sorted((p0[ax], p1[ax]))
            for plane in range(int(np.floor(lo)) + 1, int(np.ceil(hi))):
                ts.append((plane - p0[ax]) / d[ax])
    ts = np.unique(np.clip(ts, 0.0, 1.0))
    length = float(np.linalg.norm(d)) * dx
    tau = 0.0
    for a, b in zip(ts[:-1], ts[1:]):
        if b > a:
            i, j, k = np.floor(p0 + 0.5 * (a + b) * d).astype(int)
            tau += kappa[k, j, i] * (b - a) * length
    return tau


def ray_field(nH, sigma_n, c):
    """N_ray for every cell beyond 3 cells of the source, with r / dx."""
    kappa = sigma_n * nH
    out = {}
    for k in range(N_CELLS):
        for j in range(N_CELLS):
            for i in range(N_CELLS):
                r = np.sqrt((i - SRC[0]) ** 2 + (j - SRC[1]) ** 2 + (k - SRC[2]) ** 2)
                if r > 3.0:
                    tau = siddon_tau(SRC, (i, j, k), kappa, DX)
                    out[(i, j, k)] = (NDOT * np.exp(-tau) / (4 * np.pi * (r * DX) ** 2 * c), r)
    return out


def steady_state(orc, nH, steps=400):
    shp = (N_CELLS,) * 3
    p = orc.make_params(shp, DX, bc=(orc.BC_OUTFLOW,) * 6, chem=orc.CHEM_FROZEN)
    g = orc.Grid(p)
    z = np.zeros(shp)
    g.set_state(N=z, Fx=z, Fy=z, Fz=z, xHI=np.ones(shp), T=np.full(shp, 1e4), nH=nH)
    g.set_sources(np.array([SRC]), np.array([NDOT]))
    g.step(DX / (3 * orc.C_LIGHT), 1, steps)
    return g.N.copy()


def test_traversal():
    rng = np.random.default_rng(0)
    kappa = np.full((N_CELLS,) * 3, 2.5e-21)
    for _ in range(50):
        a, b = rng.integers(0, N_CELLS, 3), rng.integers(0, N_CELLS, 3)
        r = np.linalg.norm(a - b) * DX
        assert siddon_tau(a, b, kappa, DX) == pytest.approx(2.5e-21 * r, rel=1e-12)
    one = np.zeros((N_CELLS,) * 3)
    one[0, 1, 1] = 1.0                    # cell (i, j, k) = (1, 1, 0)
    assert siddon_tau((0, 0, 0), (2, 2, 0), one, 1.0) == pytest.approx(np.sqrt(2.0), rel=1e-12)
    assert siddon_tau((0, 0, 0), (2, 0, 0), one, 1.0) == 0.0
    assert siddon_tau((1, 0, 0), (1, 2, 0), one, 1.0) == pytest.approx(1.0, rel=1e-12)


def check_against_rays(N, rays):
    ratios = {key: N[key[2], key[1], key[0]] / want for key, (want, _) in rays.items()}
    near = [v for key, v in ratios.items() if rays[key][1] <= 4.0]
    mid = [v for key, v in ratios.items() if 4.0 < rays[key][1] <= 7.0]
    return np.array(near), np.array(mid), np.array(list(ratios.values()))


def test_point_source_matches_ray_casting(orc):
    nH = np.full((N_CELLS,) * 3, NH0)
    N = steady_state(orc, nH)
    near, mid, every = check_against_rays(N, ray_field(nH, orc.SIGMA_N, orc.C_LIGHT))
    print(f"N/N_ray: 3-4 cells [{near.min():.3f}, {near.max():.3f}], 4-7 cells "
          f"[{mid.min():.3f}, {mid.max():.3f}], median {np.median(every):.3f}")
    assert 0.75 <= near.min() and near.max() <= 1.35
    assert 0.8 <= mid.min() and mid.max() <= 1.25
    assert abs(np.median(every) - 1.0) < 0.05


def test_dense_clump_casts_a_shadow(orc):
    nH = np.full((N_CELLS,) * 3, NH0)
    base = steady_state(orc, nH)
    nH[7:10, 7:10, 11:13] *= 50.0         # tau ~ 10 across, on the +x side
    N = steady_state(orc, nH)
    rays = ray_field(nH, orc.SIGMA_N, orc.C_LIGHT)
    behind, mirror = N[8, 8, 14], N[8, 8, 2]
    assert rays[(14, 8, 8)][0] < 1e-3 * rays[(2, 8, 8)][0]
    assert behind < 0.2 * mirror
    # off the shadow (the -x, +-y and +-z directions) the field is unchanged
    for (i, j, k) in ((2, 8, 8), (8, 14, 8), (8, 2, 8), (8, 8, 14), (8, 8, 2)):
        assert N[k, j, i] == pytest.approx(base[k, j, i], rel=0.1)
