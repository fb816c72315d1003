"""Seeded synthetic workloads for the M1 radiative-transfer step.

This module holds only input generation (grids, densities, source lists and
the per-workload constants); none of the method's arithmetic lives here.  It
is the one module that both the GPU path's tests/benchmark and the FP64
oracle's tests draw their inputs from.

The paper post-processes RAMSES snapshots (1024^3 grids of 12.5-100 Mpc/h
boxes, star particles as sources, Sec. 2.1, 2.3 and 3.1).  Those data are not
available, so the generator stands in with the same shape: a clumpy
lognormal hydrogen density on an n^3 Cartesian grid and point sources in the
densest cells, with luminosities spread over three decades.

Recipe (the same at every n, not nested):
  * white noise g0 ~ N(0, 1) from numpy PCG64(seed), float32, shape (n,n,n);
  * filtered in Fourier space by sqrt(P(k)), P(k) ~ k^-2 in grid units,
    k = 0 removed, then standardised to zero mean and unit variance;
  * nH = mean * exp(s*g - s^2/2) with s = sigma_ln = 1.5, rescaled to the
    exact mean (2e-4 cm^-3, the cosmic mean hydrogen density at z ~ 9);
  * sources: the K densest cells (ties by ascending linear index),
    luminosities 10^U(50, 53) photons/s from PCG64(seed + 1).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 2.99792458e10          # cm/s
KPC = 3.0856775814913673e21      # cm
MPC = 1e3 * KPC

SEED_DENSITY = 20100415
SEED_LUMINOSITY = 20100416

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
CHEM_FULL, CHEM_ISOTHERMAL, CHEM_OFF, CHEM_FROZEN = 0, 1, 2, 3
PREC_FP32, PREC_MIXED = 0, 1
SUB_FIXED, SUB_ADAPTIVE = 0, 1


def white_noise(n: int, seed: int = SEED_DENSITY, shape=None) -> np.ndarray:
    shape = (n, n, n) if shape is None else tuple(shape)
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape, dtype=np.float32)


def gaussian_field(n: int, seed: int = SEED_DENSITY, slope: float = -2.0,
                   device: str = "cpu", shape=None):
    """Standardised Gaussian random field with P(k) ~ k^slope (grid units).

    The noise is drawn on the host; the FFT filter runs on ``device`` (torch)
    so that the 1024^3 case is generated in seconds.  Returns a float32
    torch tensor of shape (nz, ny, nx) on ``device``."""
    import torch

    g0 = torch.from_numpy(white_noise(n, seed, shape))
    g0 = g0.to(device)
    nz, ny, nx = g0.shape
    gk = torch.fft.rfftn(g0)
    del g0
    kz = torch.fft.fftfreq(nz, device=device, dtype=torch.float32) * nz
    ky = torch.fft.fftfreq(ny, device=device, dtype=torch.float32) * ny
    kx = torch.fft.rfftfreq(nx, device=device, dtype=torch.float32) * nx
    # multiply plane by plane to keep the temporary small at 1024^3
    half = 0.5 * slope
    kyx2 = ky[:, None] ** 2 + kx[None, :] ** 2
    for iz in range(nz):
        k2 = kyx2 + kz[iz] ** 2
        amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** half, torch.zeros_like(k2))
        gk[iz] *= amp
    g = torch.fft.irfftn(gk, s=(nz, ny, nx))
    del gk
    mean = g.double().mean()
    std = (g.double() - mean).pow(2).mean().sqrt()
    g -= mean.float()
    g /= std.float()
    return g


def lognormal_density(n: int, mean: float = 2e-4, sigma_ln: float = 1.5,
                      seed: int = SEED_DENSITY, device: str = "cpu", shape=None):
    """Hydrogen number density [cm^-3], float32 torch tensor (nz, ny, nx)."""
    g = gaussian_field(n, seed, device=device, shape=shape)
    g.mul_(sigma_ln).sub_(0.5 * sigma_ln * sigma_ln).exp_()
    g.mul_(float(mean / g.double().mean()))
    return g


def densest_cells(nH, K: int) -> np.ndarray:
    """(K, 3) int32 (i, j, k) = (x, y, z) of the K densest cells; ties are
    broken by ascending linear index (x fastest)."""
    import torch

    flat = nH.reshape(-1)
    K = int(min(K, flat.numel()))
    if K == 0:
        return np.zeros((0, 3), np.int32)
    vals, _ = torch.topk(flat, K, sorted=True)
    kth = vals[-1]
    above = torch.nonzero(flat > kth).reshape(-1)
    equal = torch.nonzero(flat == kth).reshape(-1)
    idx = torch.cat([above, equal[: K - above.numel()]])
    idx, _ = torch.sort(idx)
    idx = idx.cpu().numpy().astype(np.int64)
    nz, ny, nx = nH.shape
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    return np.stack([i, j, k], axis=1).astype(np.int32)


def luminosities(K: int, seed: int = SEED_LUMINOSITY, lo: float = 50.0,
                 hi: float = 53.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return 10.0 ** rng.uniform(lo, hi, size=K)


@dataclass
class Workload:
    name: str
    n: int
    dx: float                 # proper cell size [cm]
    dt: float                 # step [s]
    steps: int
    n_sources: int
    nH_mean: float
    T0: float
    bc: tuple = (BC_PERIODIC,) * 6
    chem: int = CHEM_FULL
    prec: int = PREC_FP32
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.n ** 3


def courant_dt(dx: float, c: float = C_LIGHT) -> float:
    """Largest stable step of the unsplit 3-D explicit update, dx/(3c)."""
    return dx / (3.0 * c)


def cosmo_dx(n: int, box_mpc_h: float = 10.0, h: float = 0.7, z: float = 9.0) -> float:
    """Proper cell size of an n^3 grid over a comoving box of box_mpc_h Mpc/h."""
    return box_mpc_h / h / (1.0 + z) * MPC / n


def workload(name: str) -> Workload:
    """The five configurations: a 32^3 Stromgren test and four cosmological
    grids (128^3 ... 1024^3) of a 10 Mpc/h box at z = 9."""
    if name == "stromgren32":
        dx = 6.6 * KPC / 32
        return Workload("stromgren32", 32, dx, courant_dt(dx), 200, 1, 2e-3, 100.0,
                        bc=(BC_REFLECT, BC_OUTFLOW) * 3,
                        note="one 5e48 /s source at the corner cell; Ndot/8 "
                             "is injected because the three low faces reflect",
                        extra=dict(ndot=5e48))
    table = {"cosmo128": (128, 256, 1000, PREC_FP32),
             "cosmo256": (256, 2048, 500, PREC_MIXED),
             "cosmo512": (512, 16384, 200, PREC_MIXED),
             "cosmo1024": (1024, 131072, 200, PREC_MIXED)}
    n, K, steps, prec = table[name]
    dx = cosmo_dx(n)
    return Workload(name, n, dx, courant_dt(dx), steps, K, 2e-4, 1e4, prec=prec)


def stromgren_sources(w: Workload):
    ijk = np.zeros((1, 3), np.int32)
    return ijk, np.array([w.extra["ndot"] / 8.0])


# Subgrid clumping laws (cr_norm, cr_exp, ci_norm, ci_exp) for
# C_R = max(1, cr_norm nH^cr_exp), C_I = ci_norm nH^ci_exp (nH in cm^-3).
# Sec. 3.2.1 fits C_R ~ nH^0.7 and C_I ~ nH^0.1 ('B' trends; C_R above one
# from ~4e-3 cm^-3, C_I ~ 1 at the mean density), and reports C_R ~ nH^2.5
# with C_I = 1 for the densest cells ('A' trends); the normalisations here
# are chosen in that spirit, the paper gives them only in figures.
CLUMP_LAWS = {
    "B": (50.0, 0.7, 2.3, 0.1),
    "A": (1.0e4, 2.5, 1.0, 0.0),
}


SEED_PARTICLES = 20100418
M_SUN = 1.98892e33        # g
MYR_S = 3.15576e13        # s


def star_particles(nH, dx: float, n: int, seed: int = SEED_PARTICLES, hosts: int = 4096,
                   mass_msun: float = 5.81e4, max_age_myr: float = 30.0):
    """Seeded synthetic stellar particles standing in for a snapshot's
    (Sec. 2.3 uses the simulations' star particles, not available here):
    n particles placed uniformly inside the `hosts` densest cells of nH
    (several per cell, so cells hold duplicates), a few shifted by one box
    length to exercise the periodic wrap; ages at the snapshot uniform in
    [0, max_age] Myr, ionising lifetimes uniform in [5, 20] Myr, photons per
    stellar baryon uniform in [24000, 98000], masses mass_msun.  Returns a
    dict of float64 numpy arrays: pos (n, 3) [cm], age_next [s],
    lifetime [s], q, mass [g]."""
    import torch

    nz, ny, nx = nH.shape
    cells = densest_cells(torch.as_tensor(nH), min(hosts, int(np.prod(nH.shape))))
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = cells[rng.integers(0, len(cells), n)].astype(np.float64)
    pos = (pick + rng.random((n, 3))) * dx
    shift = rng.random(n) < 0.02
    box = np.array([nx, ny, nz], dtype=np.float64) * dx
    pos[shift] += box * rng.choice([-1.0, 1.0], (int(shift.sum()), 3))
    return dict(pos=pos,
                age_next=rng.uniform(0.0, max_age_myr, n) * MYR_S,
                lifetime=rng.uniform(5.0, 20.0, n) * MYR_S,
                q=rng.uniform(24000.0, 98000.0, n),
                mass=np.full(n, mass_msun * M_SUN))


def cosmo_inputs(w: Workload, device: str = "cpu"):
    """(nH tensor on device, ijk, ndot) of a cosmological workload."""
    nH = lognormal_density(w.n, mean=w.nH_mean, device=device)
    ijk = densest_cells(nH, w.n_sources)
    ndot = luminosities(len(ijk))
    return nH, ijk, ndot


def random_state(shape, seed: int, c: float = C_LIGHT, nmax: float = 1e-3,
                 fmax: float = 0.9, xhi_range=(1e-6, 1.0), T_range=(1e2, 5e4),
                 nH_range=(1e-5, 1e-1)):
    """A seeded admissible radiation + gas state for parity tests: N >= 0,
    |F| <= fmax * c N, log-uniform xHI, T and nH.  Returns float32 arrays
    (exactly representable for both sides)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = (nmax * rng.random(shape) ** 3).astype(np.float32)
    d = rng.standard_normal((3,) + tuple(shape))
    d /= np.linalg.norm(d, axis=0, keepdims=True) + 1e-30
    f = fmax * rng.random(shape)
    F = (d * f * c * N.astype(np.float64)).astype(np.float32)
    lo, hi = np.log10(xhi_range[0]), np.log10(xhi_range[1])
    xHI = (10.0 ** rng.uniform(lo, hi, shape)).astype(np.float32)
    T = (10.0 ** rng.uniform(np.log10(T_range[0]), np.log10(T_range[1]), shape)).astype(np.float32)
    nH = (10.0 ** rng.uniform(np.log10(nH_range[0]), np.log10(nH_range[1]), shape)).astype(np.float32)
    return dict(N=N, Fx=F[0], Fy=F[1], Fz=F[2], xHI=xHI, T=T, nH=nH)
