"""Extreme eigenvalues of the M1 flux Jacobian, for the oracle's HLL flux
(TEST INFRASTRUCTURE ONLY; shares no code with the HIP path).

Sec. 2.2: the moment equations dN/dt + div F = 0, dF/dt + c^2 div P = 0 with
P = D N, D = (1-chi)/2 I + (3chi-1)/2 n(x)n, chi(f) the closure of reduced
flux f = |F|/(cN).  Written for U = (N, F/c) as dU/dt + c dG_d(U)/dx_d = 0,
the flux along axis d is G_d = (F_d/c, P_{xd}, P_{yd}, P_{zd}); the signal
speeds of HLL are c times the smallest and largest eigenvalue of the 4x4
Jacobian dG_d/dU.  This module evaluates that Jacobian by the complex-step
derivative (exact to rounding: no difference of nearby values is taken) and
its eigenvalues with numpy, cell by cell.

Reading: an empty cell (N = 0) has no reduced flux; it takes the isotropic
values -1/sqrt(3), +1/sqrt(3), the limit of a vanishing flux.
"""

from __future__ import annotations

import numpy as np

ISO = 1.0 / np.sqrt(3.0)


def _chi(f):
    return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * np.sqrt(4.0 - 3.0 * f * f))


def _flux(U, d):
    """G_d for U = (N, w) with w = F/c; complex-analytic in U."""
    N = U[..., 0]
    w = U[..., 1:]
    u = w / N[..., None]
    f = np.sqrt((u * u).sum(-1))            # no abs: keeps the complex step
    chi = _chi(f)
    n = u / f[..., None]
    a = 0.5 * (1.0 - chi)
    b = 0.5 * (3.0 * chi - 1.0)
    P_d = N[..., None] * (b[..., None] * n[..., d:d + 1] * n)
    P_d[..., d] += N * a
    return np.concatenate([w[..., d:d + 1], P_d], -1)


def jacobian(N, w, d):
    """(..., 4, 4) Jacobian dG_d/dU at U = (N, w) (N > 0).  The complex step
    is exact to rounding only while it is far below the state it perturbs:
    it is taken relative to N (G is homogeneous of degree one in U, so the
    Jacobian depends on the reduced flux alone), also for N near the empty
    threshold of 1e-30."""
    N = np.asarray(N, np.float64)
    U = np.concatenate([N[..., None], np.asarray(w, np.float64)], -1).astype(np.complex128)
    h = 1e-20 * N
    cols = []
    for k in range(4):
        e = np.zeros(U.shape, np.complex128)
        e[..., k] = 1j * h
        cols.append(_flux(U + e, d).imag / h[..., None])
    return np.stack(cols, -1)


def eigen_extremes(N, Fx, Fy, Fz, c):
    """(..., 6): smallest and largest eigenvalue along x, y, z, in units of
    c, of every cell of the given arrays (any shape)."""
    N = np.asarray(N, np.float64)
    w = np.stack([np.asarray(Fx, np.float64), np.asarray(Fy, np.float64),
                  np.asarray(Fz, np.float64)], -1) / c
    out = np.empty(N.shape + (6,))
    out[..., 0::2] = -ISO
    out[..., 1::2] = ISO
    f = np.sqrt((w * w).sum(-1)) / np.where(N > 0, N, 1.0)
    live = (N > 0) & (f > 1e-12)
    if live.any():
        Nl, wl = N[live], w[live]
        for d in range(3):
            ev = np.linalg.eigvals(jacobian(Nl, wl, d)).real
            out[live, 2 * d] = ev.min(-1)
            out[live, 2 * d + 1] = ev.max(-1)
    return out
