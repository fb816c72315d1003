"""FP64 CPU oracle of the explicit M1 radiative-transfer step with hydrogen
photo-chemistry (Aubert & Teyssier 2010, Sec. 2.2, Sec. 2.3, Appendix A).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package to check and time the GPU library.  It
shares no code with the GPU path and never imports it.  The arithmetic lives
in ``m1_oracle.c``; this module only builds it, marshals numpy arrays and
adds the plain sums that define the global averages.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "m1_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_GIVEN = 0, 1, 2, 3
CHEM_FULL, CHEM_ISOTHERMAL, CHEM_OFF, CHEM_FROZEN = 0, 1, 2, 3
SUB_FIXED, SUB_ADAPTIVE = 0, 1
FLUX_LF, FLUX_HLL = 0, 1
NTALLY = 5   # absorbed, escaped, floor, sub-cycles, diluted by the expansion

# gray single-group constants of Sec. 2.2 and the physical constants
SIGMA_N = 2.93e-18
SIGMA_E = 2.49e-18
EGAMMA_EV = 20.27
C_LIGHT = 2.99792458e10


def build(force: bool = True) -> str:
    """Compile the oracle into ``liboracle.so`` with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("bc", ctypes.c_int32 * 6),
                ("chem", ctypes.c_int32), ("sub", ctypes.c_int32),
                ("clump", ctypes.c_int32), ("flux", ctypes.c_int32),
                ("dx", ctypes.c_double), ("c", ctypes.c_double),
                ("sigma_n", ctypes.c_double), ("sigma_e", ctypes.c_double),
                ("egamma_eV", ctypes.c_double), ("T_floor", ctypes.c_double),
                ("sub_eps", ctypes.c_double),
                ("cr_norm", ctypes.c_double), ("cr_exp", ctypes.c_double),
                ("ci_norm", ctypes.c_double), ("ci_exp", ctypes.c_double),
                ("hubble", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_chi.restype = ctypes.c_double
        L.orc_chi.argtypes = [ctypes.c_double]
        L.orc_eddington.restype = None
        L.orc_eddington.argtypes = [ctypes.c_double] * 5 + [dp]
        L.orc_rates.restype = None
        L.orc_rates.argtypes = [ctypes.c_double, dp]
        L.orc_step_flux.restype = ctypes.c_int32
        L.orc_step_flux.argtypes = [ctypes.POINTER(Params), ctypes.c_double, ctypes.c_int32] + [
            dp] * 10
        L.orc_clumping.restype = None
        L.orc_clumping.argtypes = [ctypes.POINTER(Params), ctypes.c_double, dp, dp]
        L.orc_rates_n.restype = None
        L.orc_rates_n.argtypes = [ctypes.c_int64, dp, dp]
        L.orc_chem_timescale.restype = ctypes.c_double
        L.orc_chem_timescale.argtypes = [ctypes.POINTER(Params)] + [ctypes.c_double] * 4
        L.orc_heat_per_ionisation_erg.restype = ctypes.c_double
        L.orc_heat_per_ionisation_erg.argtypes = [ctypes.POINTER(Params)]
        L.orc_chem_cell.restype = None
        L.orc_chem_cell.argtypes = [ctypes.POINTER(Params), ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_double] + [dp] * 7 + [
                                        ctypes.POINTER(ctypes.c_int32)]
        L.orc_sources_to_field.restype = None
        L.orc_sources_to_field.argtypes = [ctypes.POINTER(Params), ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int32), dp, dp]
        L.orc_fill_ghosts.restype = None
        L.orc_fill_ghosts.argtypes = [ctypes.POINTER(Params)] + [dp] * 4
        L.orc_step.restype = ctypes.c_int32
        L.orc_step.argtypes = [ctypes.POINTER(Params), ctypes.c_double,
                               ctypes.c_int32] + [dp] * 9
        L.orc_run.restype = ctypes.c_int32
        L.orc_run.argtypes = [ctypes.POINTER(Params), ctypes.c_double,
                              ctypes.c_int32, ctypes.c_int64] + [dp] * 9
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(shape, dx, bc=(0,) * 6, chem=CHEM_FULL, sub=SUB_FIXED,
                c=C_LIGHT, sigma_n=SIGMA_N, sigma_e=SIGMA_E, egamma_eV=EGAMMA_EV,
                T_floor=10.0, sub_eps=0.1, clump=None, flux=0, hubble=0.0) -> Params:
    """``shape`` is (nz, ny, nx), the numpy order of every field.  ``clump``
    is None (no subgrid clumping) or (cr_norm, cr_exp, ci_norm, ci_exp):
    C_R = max(1, cr_norm nH^cr_exp), C_I = ci_norm nH^ci_exp.  ``hubble``:
    the expansion rate H [1/s] (0: a static medium)."""
    nz, ny, nx = shape
    cl = (0.0, 0.0, 1.0, 0.0) if clump is None else tuple(float(v) for v in clump)
    return Params(nx, ny, nz, (ctypes.c_int32 * 6)(*bc), chem, sub,
                  0 if clump is None else 1, int(flux), dx, c,
                  sigma_n, sigma_e, egamma_eV, T_floor, sub_eps, *cl, float(hubble))


# ---------------------------------------------------------------- closure
def chi(f: float) -> float:
    """Levermore closure chi(f) (Sec. 2.2)."""
    return lib().orc_chi(float(f))


def eddington(N, F, c=C_LIGHT) -> np.ndarray:
    """Pressure tensor P = D N as a symmetric 3x3 matrix (Sec. 2.2)."""
    out = np.zeros(6)
    lib().orc_eddington(float(N), float(F[0]), float(F[1]), float(F[2]), c,
                        _ptr(out))
    xx, yy, zz, xy, xz, yz = out
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def clumping(params: Params, nH: float):
    """(C_R, C_I) of a cell of density nH (Sec. 3.2.1 clumping factors)."""
    cr, ci = ctypes.c_double(), ctypes.c_double()
    lib().orc_clumping(ctypes.byref(params), float(nH), ctypes.byref(cr), ctypes.byref(ci))
    return cr.value, ci.value


def rates(T: float) -> np.ndarray:
    """[alpha_B, beta, recB cooling, colex cooling, colion cooling, brems]."""
    out = np.zeros(6)
    lib().orc_rates(float(T), _ptr(out))
    return out


def rates_n(T) -> np.ndarray:
    """rates() for an array of temperatures: shape (n, 6)."""
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(-1))
    out = np.zeros((T.size, 6))
    lib().orc_rates_n(T.size, _ptr(T), _ptr(out))
    return out


def chem_timescale(params: Params, nH, N, xHI, T) -> float:
    """The adaptive sub-cycle time scale of one cell [s] (inf if static)."""
    return lib().orc_chem_timescale(ctypes.byref(params), float(nH), float(N), float(xHI),
                                    float(T))


def heat_per_ionisation_erg(params: Params) -> float:
    return lib().orc_heat_per_ionisation_erg(ctypes.byref(params))


def chem_cell(params: Params, dt, nsub, nH, N, F, xHI, T):
    """Phi on one cell.  Returns (N, F[3], xHI, T, absorbed, ncycles)."""
    v = [ctypes.c_double(float(q)) for q in (N, F[0], F[1], F[2], xHI, T, 0.0)]
    nc = ctypes.c_int32(0)
    lib().orc_chem_cell(ctypes.byref(params), float(dt), int(nsub), float(nH),
                        *[ctypes.byref(q) for q in v], ctypes.byref(nc))
    return (v[0].value, np.array([v[1].value, v[2].value, v[3].value]),
            v[4].value, v[5].value, v[6].value, nc.value)


# ---------------------------------------------------------------- grid
class Grid:
    """FP64 state on the host.  Public fields are interior (nz, ny, nx) views;
    N and F live in padded arrays with a one-cell ghost layer."""

    def __init__(self, params: Params):
        self.p = params
        nz, ny, nx = params.nz, params.ny, params.nx
        pad = (nz + 2, ny + 2, nx + 2)
        self._U = [np.zeros(pad) for _ in range(4)]
        self.xHI = np.ones((nz, ny, nx))
        self.T = np.full((nz, ny, nx), 1e4)
        self.nH = np.full((nz, ny, nx), 1e-3)
        self.S = np.zeros((nz, ny, nx))
        self.tally = np.zeros(NTALLY)  # absorbed, escaped, floor, sub-cycles, diluted
        self.emitted = 0.0
        self.t = 0.0
        self.nsrc_rate = 0.0      # sum of Ndot of the current sources

    @property
    def shape(self):
        return (self.p.nz, self.p.ny, self.p.nx)

    def _interior(self, a):
        return a[1:-1, 1:-1, 1:-1]

    @property
    def N(self):
        return self._interior(self._U[0])

    @property
    def Fx(self):
        return self._interior(self._U[1])

    @property
    def Fy(self):
        return self._interior(self._U[2])

    @property
    def Fz(self):
        return self._interior(self._U[3])

    def padded(self, m):
        """Padded array m (0 N, 1 Fx, 2 Fy, 3 Fz), ghosts writable."""
        return self._U[m]

    def set_state(self, N=None, Fx=None, Fy=None, Fz=None, xHI=None, T=None,
                  nH=None):
        for m, a in enumerate((N, Fx, Fy, Fz)):
            if a is not None:
                self._interior(self._U[m])[...] = a
        if xHI is not None:
            self.xHI[...] = xHI
        if T is not None:
            self.T[...] = T
        if nH is not None:
            self.nH[...] = nH

    def set_sources(self, ijk, ndot):
        """Replace the point sources: ijk (n, 3) int as (i, j, k) = (x, y, z)."""
        ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
        ndot = np.ascontiguousarray(np.asarray(ndot, dtype=np.float64).reshape(-1))
        self.S[...] = 0.0
        if len(ndot):
            lib().orc_sources_to_field(
                ctypes.byref(self.p), len(ndot),
                ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(ndot),
                _ptr(self.S))
        self.nsrc_rate = float(np.sum(ndot))

    def _lam(self):
        """Per padded cell extreme Jacobian eigenvalues (HLL), ghosts filled."""
        from . import hll
        self.fill_ghosts()
        return np.ascontiguousarray(hll.eigen_extremes(*self._U, self.p.c))

    def step(self, dt, nsub=1, nsteps=1):
        if self.p.flux == FLUX_HLL:
            acc = np.zeros(NTALLY)
            for _ in range(int(nsteps)):
                lam = self._lam()
                tl = np.zeros(NTALLY)
                rc = lib().orc_step_flux(ctypes.byref(self.p), float(dt), int(nsub),
                                         *[_ptr(u) for u in self._U], _ptr(self.xHI),
                                         _ptr(self.T), _ptr(self.nH), _ptr(self.S), _ptr(lam),
                                         _ptr(tl))
                if rc != 0:
                    raise ValueError(f"orc_step_flux failed with {rc}")
                acc += tl
            self.tally += acc
            self.emitted += self.nsrc_rate * dt * nsteps
            self.t += dt * nsteps
            return acc
        tl = np.zeros(NTALLY)
        rc = lib().orc_run(ctypes.byref(self.p), float(dt), int(nsub), int(nsteps),
                           *[_ptr(u) for u in self._U], _ptr(self.xHI),
                           _ptr(self.T), _ptr(self.nH), _ptr(self.S), _ptr(tl))
        if rc != 0:
            raise ValueError(f"orc_run failed with {rc}")
        self.tally += tl
        self.emitted += self.nsrc_rate * dt * nsteps
        self.t += dt * nsteps
        return tl

    def fill_ghosts(self):
        lib().orc_fill_ghosts(ctypes.byref(self.p), *[_ptr(u) for u in self._U])

    # ------------------------------------------------- global averages
    def reductions(self) -> dict:
        """Volume- and mass-weighted neutral fraction (Sec. 3.1.1-3.1.2), the
        volume-averaged photoionisation rate c sigma_n N (Sec. 3.1.3) and the
        photon budget, all as plain FP64 sums."""
        vol = self.p.dx ** 3
        ncell = self.N.size
        stored = float(np.sum(self.N)) * vol
        return dict(
            t=self.t,
            xhi_vol=float(np.sum(self.xHI)) / ncell,
            xhi_mass=float(np.sum(self.nH * self.xHI)) / float(np.sum(self.nH)),
            gamma_vol=self.p.c * self.p.sigma_n * float(np.sum(self.N)) / ncell,
            photons_emitted=self.emitted,
            photons_stored=stored,
            photons_absorbed=float(self.tally[0]),
            photons_escaped=float(self.tally[1]),
            photons_floor=float(self.tally[2]),
            photons_diluted=float(self.tally[4]),
        )


def step_subblock(params: Params, dt, nsub, Npad, Fpad, xHI, T, nH, S=None):
    """One step of an interior sub-block whose one-cell halo is supplied by
    the caller (every face ORC_BC_GIVEN).  Npad (nz+2, ny+2, nx+2); Fpad a
    list of three such arrays; xHI, T, nH, S (nz, ny, nx).  Returns the
    stepped interior (N, Fx, Fy, Fz, xHI, T, tally)."""
    p = Params.from_buffer_copy(params)
    for f in range(6):
        p.bc[f] = BC_GIVEN
    p.nz, p.ny, p.nx = np.shape(xHI)
    for a in [Npad] + list(Fpad):
        if np.shape(a) != (p.nz + 2, p.ny + 2, p.nx + 2):
            raise ValueError("padded arrays must be (nz+2, ny+2, nx+2)")
    for a in (T, nH) + (() if S is None else (S,)):
        if np.shape(a) != (p.nz, p.ny, p.nx):
            raise ValueError("xHI, T, nH, S must share one shape")
    U = [np.ascontiguousarray(Npad, dtype=np.float64)] + [
        np.ascontiguousarray(a, dtype=np.float64) for a in Fpad]
    xHI = np.ascontiguousarray(xHI, dtype=np.float64).copy()
    T = np.ascontiguousarray(T, dtype=np.float64).copy()
    nH = np.ascontiguousarray(nH, dtype=np.float64)
    S = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
    U = [u.copy() for u in U]
    tl = np.zeros(NTALLY)
    if p.flux == FLUX_HLL:
        from . import hll
        lam = np.ascontiguousarray(hll.eigen_extremes(*U, p.c))
        rc = lib().orc_step_flux(ctypes.byref(p), float(dt), int(nsub), *[_ptr(u) for u in U],
                                 _ptr(xHI), _ptr(T), _ptr(nH), _ptr(S), _ptr(lam), _ptr(tl))
    else:
        rc = lib().orc_step(ctypes.byref(p), float(dt), int(nsub), *[_ptr(u) for u in U],
                            _ptr(xHI), _ptr(T), _ptr(nH), _ptr(S), _ptr(tl))
    if rc != 0:
        raise ValueError(f"orc_step failed with {rc}")
    inner = tuple(u[1:-1, 1:-1, 1:-1].copy() for u in U)
    return inner + (xHI, T, tl)
