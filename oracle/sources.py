"""FP64 reference of the source pipeline (TEST INFRASTRUCTURE ONLY: loaded by
the tests and nothing else; shares no code with the HIP path).

Sec. 2.3: the sources are stellar particles of the hydrodynamical snapshots.
Each has an ionising lifetime L (drawn between 5 and 20 Myr) and emits, over
that lifetime, Q ionising photons per stellar baryon (between 24000 and
98000), i.e. at the intrinsic rate Ndot = Q (m / m_b) / L while its age lies
in [0, L].  Between snapshots p and p+1 (times t_p < t_{p+1}, Delta = t_{p+1}
- t_p) only the particles of snapshot p+1 are used; with age a_{p+1} there,
a_p = a_{p+1} - Delta.  The photons a particle emits within the interval,
Ndot times the overlap of its emitting ages [0, L] with [a_p, a_{p+1}], are
spread evenly over the interval (the paper's 'diluted' rate):

    rate = Ndot * max(0, min(a_{p+1}, L) - max(a_p, 0)) / Delta

which is zero when a_p >= L, min(a_{p+1}, L) / Delta * Ndot for a particle
born within the interval (a_p < 0) and min(Delta, L - a_p) / Delta * Ndot
otherwise.  The effective rate is rate * f_esc * B(t) with the boost factor
B(t) = max(1, a_b exp(k_b / t)), t the age of the Universe, taken here at
the middle of the interval.  Particles are assigned to the cell holding
them (nearest grid point, periodic box), each cell one source, duplicate
cells summed.
"""

from __future__ import annotations

import math

import numpy as np

M_BARYON = 1.67262192e-24   # g (proton mass)
MYR = 3.15576e13            # s (Julian Myr)


def emitting_overlap(age_next, lifetime, delta):
    """Length of [max(a_p, 0), min(a_{p+1}, L)] (zero if empty), a_p =
    a_{p+1} - delta."""
    age_next = np.asarray(age_next, dtype=np.float64)
    lifetime = np.asarray(lifetime, dtype=np.float64)
    a_p = age_next - delta
    return np.maximum(0.0, np.minimum(age_next, lifetime) - np.maximum(a_p, 0.0))


def intrinsic_rate(q_per_baryon, mass_g, lifetime):
    """Ndot = Q m / (m_b L) [photons / s]."""
    return (np.asarray(q_per_baryon, dtype=np.float64) * np.asarray(mass_g, dtype=np.float64)
            / M_BARYON / np.asarray(lifetime, dtype=np.float64))


def boost(t, a_b, k_b):
    """B(t) = max(1, a_b exp(k_b / t)), exp from the host libm."""
    return max(1.0, a_b * math.exp(k_b / t))


def particle_rates(age_next, lifetime, q_per_baryon, mass_g, t_p, t_next, f_esc, a_b, k_b):
    """Effective, diluted emission rate of every particle over [t_p, t_next]."""
    delta = t_next - t_p
    Ndot = intrinsic_rate(q_per_baryon, mass_g, lifetime)
    dil = emitting_overlap(age_next, lifetime, delta) / delta
    return Ndot * dil * f_esc * boost(0.5 * (t_p + t_next), a_b, k_b)


def ngp_cells(pos_cm, dx, shape):
    """(n, 3) positions [cm] -> (n, 3) cell indices (i, j, k) = floor(pos /
    dx) wrapped into the periodic box; shape = (nz, ny, nx)."""
    nz, ny, nx = shape
    ijk = np.floor(np.asarray(pos_cm, dtype=np.float64) / dx).astype(np.int64)
    ijk[:, 0] %= nx
    ijk[:, 1] %= ny
    ijk[:, 2] %= nz
    return ijk


def source_field(ijk, rates, shape):
    """Dense (nz, ny, nx) field of summed rates per cell [photons / s]."""
    S = np.zeros(shape, dtype=np.float64)
    np.add.at(S, (ijk[:, 2], ijk[:, 1], ijk[:, 0]), np.asarray(rates, dtype=np.float64))
    return S
