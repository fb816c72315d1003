"""ctypes binding of librt_m1.so (include/rt.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The functions carry the C names (rt_init, rt_inject_sources,
rt_step, rt_reduce, rt_state, rt_current, rt_profile, rt_profile_read,
rt_destroy, rt_strerror); ``RTGrid`` is a convenience owner of the torch
device tensors that the library borrows.  Loading fails loudly if the library
has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_m1.so")

RT_OK, RT_E_ARG, RT_E_CFL, RT_E_STATE, RT_E_HIP, RT_E_NONFINITE, RT_E_NOMEM = (
    0, -1, -2, -3, -4, -5, -6)
RT_E_SCRATCH = -7
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
CHEM_FULL, CHEM_ISOTHERMAL, CHEM_OFF, CHEM_FROZEN = 0, 1, 2, 3
PREC_FP32, PREC_MIXED = 0, 1
SUB_FIXED, SUB_ADAPTIVE = 0, 1
FLUX_LF, FLUX_HLL = 0, 1
FIELD_N, FIELD_FX, FIELD_FY, FIELD_FZ, FIELD_XHI, FIELD_T, FIELD_NH = range(7)

SIGMA_N = 2.93e-18
SIGMA_E = 2.49e-18
EGAMMA_EV = 20.27
C_LIGHT = 2.99792458e10

_fp = ctypes.c_void_p


class rt_fields(ctypes.Structure):
    _fields_ = [("N", _fp * 2), ("Fx", _fp * 2), ("Fy", _fp * 2), ("Fz", _fp * 2),
                ("xHI", _fp), ("T", _fp), ("nH", _fp)]


class rt_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 6), ("chem", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("sub", ctypes.c_int32),
                ("clump", ctypes.c_int32), ("flux", ctypes.c_int32),
                ("dx_cm", ctypes.c_double), ("c_cms", ctypes.c_double),
                ("sigma_n", ctypes.c_double), ("sigma_e", ctypes.c_double),
                ("egamma_eV", ctypes.c_double), ("T_floor", ctypes.c_double),
                ("sub_eps", ctypes.c_double), ("xhi_fp64_thr", ctypes.c_double),
                ("clump_cr_norm", ctypes.c_double), ("clump_cr_exp", ctypes.c_double),
                ("clump_ci_norm", ctypes.c_double), ("clump_ci_exp", ctypes.c_double)]


class rt_reductions(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("xhi_vol", ctypes.c_double),
                ("xhi_mass", ctypes.c_double), ("gamma_vol", ctypes.c_double),
                ("photons_initial", ctypes.c_double), ("photons_emitted", ctypes.c_double),
                ("photons_stored", ctypes.c_double), ("photons_absorbed", ctypes.c_double),
                ("photons_escaped", ctypes.c_double), ("photons_floor", ctypes.c_double),
                ("steps", ctypes.c_int64), ("n_nonfinite", ctypes.c_int64),
                ("n_fp64", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("subcycle_hist", ctypes.c_int64 * 8), ("tau_e", ctypes.c_double),
                ("n_learned", ctypes.c_int64), ("n_fallback_range", ctypes.c_int64),
                ("photons_diluted", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "subcycle_hist"}
        d["subcycle_hist"] = list(self.subcycle_hist)
        return d


EXPORTS = ["rt_init", "rt_inject_sources", "rt_step", "rt_reduce", "rt_state",
           "rt_current", "rt_profile", "rt_profile_read", "rt_destroy", "rt_strerror",
           "rt_histogram", "rt_set_expansion"]

HQ_XHI, HQ_GAMMA = 0, 1
HIST_MAX_BINS = 8192

_lib = None


class RTError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {rt_strerror(code)} ({code})")
        self.code = code


def lib():
    """Load librt_m1.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1004_2503_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.rt_init.argtypes = [P(rt_params), P(rt_fields), vp, P(vp)]
        L.rt_inject_sources.argtypes = [vp, ctypes.c_int64, P(ctypes.c_int32),
                                        P(ctypes.c_double)]
        L.rt_step.argtypes = [vp, ctypes.c_double, ctypes.c_int32]
        L.rt_set_expansion.argtypes = [vp, ctypes.c_double]
        L.rt_reduce.argtypes = [vp, P(rt_reductions)]
        L.rt_state.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32]
        L.rt_current.argtypes = [vp, P(ctypes.c_int32)]
        L.rt_profile.argtypes = [vp, ctypes.c_int32]
        L.rt_profile_read.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int64)]
        L.rt_destroy.argtypes = [vp]
        L.rt_histogram.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_double, P(ctypes.c_int64), P(ctypes.c_double)]
        L.rt_strerror.argtypes = [ctypes.c_int]
        L.rt_strerror.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "rt_strerror":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


# ------------------------------------------------------------ C names
def rt_strerror(code: int) -> str:
    return lib().rt_strerror(int(code)).decode()


def rt_init(params: rt_params, fields: rt_fields, stream: int | None):
    """Returns (code, ctx handle)."""
    ctx = ctypes.c_void_p()
    rc = lib().rt_init(ctypes.byref(params), ctypes.byref(fields),
                       ctypes.c_void_p(stream or 0), ctypes.byref(ctx))
    return rc, ctx


def rt_inject_sources(ctx, ijk, ndot) -> int:
    ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    ndot = np.ascontiguousarray(np.asarray(ndot, dtype=np.float64).reshape(-1))
    if len(ijk) != len(ndot):
        return RT_E_ARG
    return lib().rt_inject_sources(
        ctx, len(ndot), ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        ndot.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def rt_step(ctx, dt: float, nsub: int) -> int:
    return lib().rt_step(ctx, float(dt), int(nsub))


def rt_set_expansion(ctx, hubble: float) -> int:
    return lib().rt_set_expansion(ctx, float(hubble))


def rt_reduce(ctx):
    out = rt_reductions()
    rc = lib().rt_reduce(ctx, ctypes.byref(out))
    return rc, out


def rt_histogram(ctx, quantity: int, xrange, yrange):
    """Returns (code, counts (nbx, nby) int64, sums (nbx,) float64);
    xrange = (lo, hi, nb) in log10 nH, yrange = (lo, hi, nb) in log10 q."""
    lox, hix, nbx = xrange
    loy, hiy, nby = yrange
    counts = np.zeros((max(int(nbx), 0), max(int(nby), 0)), np.int64)
    sums = np.zeros(max(int(nbx), 0), np.float64)
    rc = lib().rt_histogram(ctx, int(quantity), int(nbx), float(lox), float(hix), int(nby),
                            float(loy), float(hiy),
                            counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            sums.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, counts, sums


def rt_state(ctx, field: int, dst_ptr: int, on_device: bool) -> int:
    return lib().rt_state(ctx, int(field), ctypes.c_void_p(dst_ptr), int(bool(on_device)))


def rt_current(ctx):
    idx = ctypes.c_int32()
    rc = lib().rt_current(ctx, ctypes.byref(idx))
    return rc, idx.value


def rt_profile(ctx, enable: bool) -> int:
    return lib().rt_profile(ctx, int(bool(enable)))


def rt_profile_read(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    rc = lib().rt_profile_read(ctx, ctypes.byref(ms), ctypes.byref(n))
    return rc, ms.value, n.value


def rt_destroy(ctx) -> int:
    return lib().rt_destroy(ctx)


def check(rc: int, what: str):
    if rc != RT_OK:
        raise RTError(rc, what)


def make_params(shape, dx, bc=(BC_PERIODIC,) * 6, chem=CHEM_FULL, prec=PREC_FP32,
                sub=SUB_FIXED, c=C_LIGHT, T_floor=10.0, sub_eps=0.1,
                xhi_fp64_thr=1e-3, clump=None, flux=FLUX_LF) -> rt_params:
    """``shape`` is (nz, ny, nx), the torch/numpy order of every field.
    ``clump`` is None (no subgrid clumping) or (cr_norm, cr_exp, ci_norm,
    ci_exp): C_R = max(1, cr_norm nH^cr_exp), C_I = ci_norm nH^ci_exp.
    ``flux`` is FLUX_LF (the paper's Lax-Friedrichs) or FLUX_HLL."""
    nz, ny, nx = shape
    cl = (1.0, 0.0, 1.0, 0.0) if clump is None else tuple(float(v) for v in clump)
    return rt_params(nx, ny, nz, (ctypes.c_int32 * 6)(*bc), chem, prec, sub,
                     0 if clump is None else 1, int(flux),
                     float(dx), float(c), SIGMA_N, SIGMA_E, EGAMMA_EV, float(T_floor),
                     float(sub_eps), float(xhi_fp64_thr), *cl)


NFIELD_BUFFERS = 11      # N, Fx, Fy, Fz twice, xHI, T, nH
FIELD_STAGGER = 64       # floats (256 bytes) between the fields' channel offsets


class RTGrid:
    """Torch-owned device fields bound to one library context.

    ``state`` is a dict of (nz, ny, nx) arrays or tensors: N, Fx, Fy, Fz,
    xHI, T, nH (missing N/F start at zero)."""

    def __init__(self, params: rt_params, state: dict, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.params = params
        shape = (params.nz, params.ny, params.nx)
        self.shape = shape
        self.device = torch.device(device)

        # The eleven fields are views of one allocation, field k starting
        # k * FIELD_STAGGER floats past a 256-byte-aligned stride, so that
        # the streams of one cell index fall on different HBM channels.
        ncell = shape[0] * shape[1] * shape[2]
        stride = (ncell + 63) // 64 * 64 + FIELD_STAGGER
        self._slab = torch.empty(stride * (NFIELD_BUFFERS - 1) + ncell, dtype=torch.float32,
                                 device=self.device)
        slots = iter(range(NFIELD_BUFFERS))

        def dev(name, fill=0.0):
            k = next(slots)
            t = self._slab[k * stride:k * stride + ncell].view(shape)
            v = state.get(name) if name else None
            if v is None:
                t.fill_(fill)
            else:
                t.copy_(torch.as_tensor(v).to(device=self.device,
                                              dtype=torch.float32).reshape(shape))
            return t

        self.N = [dev("N"), dev(None)]
        self.Fx = [dev("Fx"), dev(None)]
        self.Fy = [dev("Fy"), dev(None)]
        self.Fz = [dev("Fz"), dev(None)]
        self.xHI = dev("xHI", 1.0)
        self.T = dev("T", 1e4)
        self.nH = dev("nH", 1e-3)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        f = rt_fields()
        f.N[0], f.N[1] = self.N[0].data_ptr(), self.N[1].data_ptr()
        f.Fx[0], f.Fx[1] = self.Fx[0].data_ptr(), self.Fx[1].data_ptr()
        f.Fy[0], f.Fy[1] = self.Fy[0].data_ptr(), self.Fy[1].data_ptr()
        f.Fz[0], f.Fz[1] = self.Fz[0].data_ptr(), self.Fz[1].data_ptr()
        f.xHI, f.T, f.nH = self.xHI.data_ptr(), self.T.data_ptr(), self.nH.data_ptr()
        self.fields = f
        torch.cuda.synchronize(self.device)
        rc, self.ctx = rt_init(params, f, self.stream.cuda_stream)
        check(rc, "rt_init")

    def inject_sources(self, ijk, ndot):
        check(rt_inject_sources(self.ctx, ijk, ndot), "rt_inject_sources")

    def step(self, dt, nsub=1, nsteps=1):
        for _ in range(int(nsteps)):
            check(rt_step(self.ctx, dt, nsub), "rt_step")

    def set_expansion(self, hubble: float):
        check(rt_set_expansion(self.ctx, hubble), "rt_set_expansion")

    def reduce(self, allow_nonfinite=False) -> dict:
        rc, out = rt_reduce(self.ctx)
        if not (rc == RT_OK or (allow_nonfinite and rc == RT_E_NONFINITE)):
            raise RTError(rc, "rt_reduce")
        return out.as_dict()

    def current(self) -> int:
        rc, idx = rt_current(self.ctx)
        check(rc, "rt_current")
        return idx

    def tensors(self) -> dict:
        """Current-state device tensors (views, no copy); waits for the stream."""
        self.stream.synchronize()
        c = self.current()
        return dict(N=self.N[c], Fx=self.Fx[c], Fy=self.Fy[c], Fz=self.Fz[c],
                    xHI=self.xHI, T=self.T, nH=self.nH)

    def state_numpy(self) -> dict:
        """Current state copied to host through rt_state."""
        out = {}
        for name, fid in (("N", FIELD_N), ("Fx", FIELD_FX), ("Fy", FIELD_FY),
                          ("Fz", FIELD_FZ), ("xHI", FIELD_XHI), ("T", FIELD_T),
                          ("nH", FIELD_NH)):
            a = np.empty(self.shape, np.float32)
            check(rt_state(self.ctx, fid, a.ctypes.data, False), "rt_state")
            out[name] = a
        return out

    def sources_from_particles(self, parts: dict, t_p, t_next, f_esc, a_b, k_b) -> int:
        """Replace the sources by those of a particle set (dict of float64
        device tensors pos, age_next, lifetime, q, mass); returns the number
        of emitting particles."""
        rc, m = rt_sources_from_particles(self.ctx, parts["pos"], parts["age_next"],
                                          parts["lifetime"], parts["q"], parts["mass"], t_p,
                                          t_next, f_esc, a_b, k_b)
        check(rc, "rt_sources_from_particles")
        return m

    def gamma_plateau(self, nH_max: float):
        """(gamma0, ncells): mean photoionisation rate below nH_max."""
        rc, g, n = rt_gamma_plateau(self.ctx, nH_max)
        check(rc, "rt_gamma_plateau")
        return g, n

    def histogram(self, quantity: int, xrange, yrange):
        """(counts, per-density-bin sums) of the current state, see rt_histogram."""
        rc, counts, sums = rt_histogram(self.ctx, quantity, xrange, yrange)
        check(rc, "rt_histogram")
        return counts, sums

    def profile(self, enable: bool):
        check(rt_profile(self.ctx, enable), "rt_profile")

    def profile_read(self):
        rc, ms, n = rt_profile_read(self.ctx)
        check(rc, "rt_profile_read")
        return ms, n

    def close(self):
        if self.ctx is not None and self.ctx.value:
            check(rt_destroy(self.ctx), "rt_destroy")
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------ batch chemistry and MLP
MLP_NPARAM = 8834
MLP_NOALLOC_BLOCKS = 256
EXPORTS += ["rt_chem_apply", "rt_mlp_create", "rt_mlp_forward", "rt_mlp_grad", "rt_mlp_adam",
            "rt_mlp_destroy", "rt_mlp_grad_noalloc", "rt_mlp_pairs", "rt_mlp_standardize",
            "rt_mlp_train", "rt_mlp_predict"]


class rt_mlp_train_opts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int64), ("total_steps", ctypes.c_int64),
                ("lr", ctypes.c_double), ("warmup", ctypes.c_double),
                ("lr_floor", ctypes.c_double), ("clip", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("seed", ctypes.c_uint64)]


def _bind_extra(L):
    vp = ctypes.c_void_p
    if getattr(L, "_extra_bound", False):
        return L
    L.rt_chem_apply.argtypes = [ctypes.POINTER(rt_params), ctypes.c_int64, vp, vp, vp, vp, vp,
                                ctypes.c_int32, vp, vp]
    L.rt_mlp_create.argtypes = [ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.rt_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
    L.rt_mlp_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, vp]
    L.rt_mlp_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.rt_mlp_destroy.argtypes = [vp]
    L.rt_mlp_grad_noalloc.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int64, vp, vp, vp]
    L.rt_mlp_pairs.argtypes = [ctypes.POINTER(rt_params), ctypes.c_int64, vp, vp, vp, vp, vp,
                               ctypes.c_int32, vp, vp, vp, vp, vp]
    L.rt_mlp_standardize.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp]
    L.rt_mlp_train.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int64,
                               ctypes.POINTER(rt_mlp_train_opts), ctypes.c_int64,
                               ctypes.c_int64, vp]
    L.rt_mlp_predict.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float), vp, ctypes.c_int64,
                                 vp, vp, vp]
    for n in ("rt_chem_apply", "rt_mlp_create", "rt_mlp_forward", "rt_mlp_grad",
              "rt_mlp_adam", "rt_mlp_destroy", "rt_mlp_grad_noalloc", "rt_mlp_pairs",
              "rt_mlp_standardize", "rt_mlp_train", "rt_mlp_predict"):
        getattr(L, n).restype = ctypes.c_int
    L._extra_bound = True
    return L


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def rt_chem_apply(params: rt_params, nH, N, xHI, T, dt, nsub: int, ncycles=None,
                  stream: int | None = None) -> int:
    """Phi on a batch of cells: torch float32 device tensors, updated in place."""
    L = _bind_extra(lib())
    n = int(nH.numel())
    for t in (N, xHI, T, dt):
        if t.numel() != n:
            return RT_E_ARG
    return L.rt_chem_apply(ctypes.byref(params), n, _p(nH), _p(N), _p(xHI), _p(T), _p(dt),
                           int(nsub), _p(ncycles), ctypes.c_void_p(stream or 0))


def rt_mlp_create(grad_blocks: int, stream: int | None = None):
    L = _bind_extra(lib())
    h = ctypes.c_void_p()
    rc = L.rt_mlp_create(int(grad_blocks), ctypes.c_void_p(stream or 0), ctypes.byref(h))
    return rc, h


def rt_mlp_forward(m, theta, X, Y) -> int:
    return _bind_extra(lib()).rt_mlp_forward(m, _p(theta), _p(X), int(X.shape[0]), _p(Y))


def rt_mlp_grad(m, theta, X, Y, grad, loss_dev=None) -> int:
    return _bind_extra(lib()).rt_mlp_grad(m, _p(theta), _p(X), _p(Y), int(X.shape[0]),
                                          _p(grad), _p(loss_dev))


def rt_mlp_grad_noalloc(grad_blocks: int, theta, X, Y, grad, loss_dev=None,
                        stream: int | None = None) -> int:
    n = 0 if X is None else int(X.shape[0])
    return _bind_extra(lib()).rt_mlp_grad_noalloc(int(grad_blocks), _p(theta), _p(X), _p(Y), n,
                                                  _p(grad), _p(loss_dev),
                                                  ctypes.c_void_p(stream or 0))


def rt_mlp_adam(m, theta, mom1, mom2, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8) -> int:
    return _bind_extra(lib()).rt_mlp_adam(m, _p(theta), _p(mom1), _p(mom2), _p(grad), int(step),
                                          float(lr), float(beta1), float(beta2), float(eps))


def rt_mlp_destroy(m) -> int:
    return _bind_extra(lib()).rt_mlp_destroy(m)


def rt_mlp_pairs(params: rt_params, nH, N, xHI, T, dt, nsub: int, X=None, U=None, Yend=None,
                 ncycles=None, stream: int | None = None) -> int:
    """Features X (n, 5), encoded targets U (n, 2), end values Yend (n, 2)
    of n cells: torch float32 device tensors (outputs preallocated or None)."""
    L = _bind_extra(lib())
    n = int(nH.numel())
    for t in (N, xHI, T, dt):
        if t.numel() != n:
            return RT_E_ARG
    for t, w in ((X, 5), (U, 2), (Yend, 2), (ncycles, 1)):
        if t is not None and t.numel() != n * w:
            return RT_E_ARG
    return L.rt_mlp_pairs(ctypes.byref(params), n, _p(nH), _p(N), _p(xHI), _p(T), _p(dt),
                          int(nsub), _p(X), _p(U), _p(Yend), _p(ncycles),
                          ctypes.c_void_p(stream or 0))


def rt_mlp_standardize(m, A, out, stats) -> int:
    """A, out: (n, d) float32 device tensors; stats: (4 d,) float64 device."""
    n, d = (int(A.shape[0]), int(A.shape[1]))
    if out.shape != A.shape or stats.numel() != 4 * d:
        return RT_E_ARG
    return _bind_extra(lib()).rt_mlp_standardize(m, _p(A), n, d, _p(out), _p(stats))


def rt_mlp_train(m, theta, mom1, mom2, X, Y, opts: rt_mlp_train_opts, step0: int, nsteps: int,
                 loss_dev=None) -> int:
    if X.shape[0] != Y.shape[0]:
        return RT_E_ARG
    return _bind_extra(lib()).rt_mlp_train(m, _p(theta), _p(mom1), _p(mom2), _p(X), _p(Y),
                                           int(X.shape[0]), ctypes.byref(opts), int(step0),
                                           int(nsteps), _p(loss_dev))


def rt_mlp_predict(m, theta, norm, X, Y=None, U=None, loss_dev=None) -> int:
    """norm: 14 host floats (mu_in, sd_in, mu_out, sd_out)."""
    nm = (ctypes.c_float * 14)(*[float(v) for v in norm[:14]])
    return _bind_extra(lib()).rt_mlp_predict(m, _p(theta), nm, _p(X), int(X.shape[0]), _p(Y),
                                             _p(U), _p(loss_dev))


EXPORTS += ["rt_set_surrogate", "rt_sources_from_particles"]


def rt_sources_from_particles(ctx, pos, age_next, lifetime, q_per_baryon, mass_g, t_p: float,
                              t_next: float, f_esc: float, a_b: float, k_b: float):
    """Particles as float64 device tensors (pos (n, 3) in cm, the rest (n,)).
    Returns (code, number of emitting particles)."""
    L = lib()
    vp = ctypes.c_void_p
    L.rt_sources_from_particles.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp] + [
        ctypes.c_double] * 5 + [ctypes.POINTER(ctypes.c_int64)]
    L.rt_sources_from_particles.restype = ctypes.c_int
    n = int(age_next.numel())
    for t in (lifetime, q_per_baryon, mass_g):
        if t.numel() != n:
            return RT_E_ARG, 0
    if pos.numel() != 3 * n:
        return RT_E_ARG, 0
    out = ctypes.c_int64(0)
    rc = L.rt_sources_from_particles(ctx, n, _p(pos), _p(age_next), _p(lifetime),
                                     _p(q_per_baryon), _p(mass_g), float(t_p), float(t_next),
                                     float(f_esc), float(a_b), float(k_b), ctypes.byref(out))
    return rc, out.value


def rt_set_surrogate(ctx, theta, norm, residual_tol: float) -> int:
    """theta: torch float32 device tensor (8834) or None (off); norm: 24 host
    floats (mu_in, sd_in, mu_out, sd_out, in_min, in_max)."""
    L = lib()
    L.rt_set_surrogate.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_float), ctypes.c_double]
    L.rt_set_surrogate.restype = ctypes.c_int
    if theta is None:
        return L.rt_set_surrogate(ctx, None, None, 0.0)
    nv = np.ascontiguousarray(np.asarray(norm, dtype=np.float32).reshape(-1))
    if nv.size != 24:
        return RT_E_ARG
    return L.rt_set_surrogate(ctx, ctypes.c_void_p(theta.data_ptr()),
                              nv.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                              float(residual_tol))


EXPORTS += ["rt_equilibrium_xhi"]
JMODEL_UNIFORM, JMODEL_EXP1, JMODEL_EXP4 = 0, 1, 2


def rt_equilibrium_xhi(params: rt_params, model: int, gamma0: float, n_star: float, nH, T, xhi,
                       stream: int | None = None) -> int:
    """Equilibrium neutral fraction under a self-shielding model (torch
    float64 device tensors of one size); asynchronous on ``stream``."""
    L = lib()
    vp = ctypes.c_void_p
    L.rt_equilibrium_xhi.argtypes = [ctypes.POINTER(rt_params), ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp]
    L.rt_equilibrium_xhi.restype = ctypes.c_int
    n = int(nH.numel())
    if T.numel() != n or xhi.numel() != n:
        return RT_E_ARG
    return L.rt_equilibrium_xhi(ctypes.byref(params), int(model), float(gamma0), float(n_star),
                                n, _p(nH), _p(T), _p(xhi), vp(stream or 0))


def equilibrium_xhi(params: rt_params, model: int, gamma0: float, n_star: float, nH, T):
    """New float64 tensor of equilibrium neutral fractions (see
    rt_equilibrium_xhi); nH and T are float64 device tensors."""
    import torch

    out = torch.empty_like(nH)
    check(rt_equilibrium_xhi(params, model, gamma0, n_star, nH, T, out,
                             torch.cuda.current_stream(nH.device).cuda_stream),
          "rt_equilibrium_xhi")
    return out


EXPORTS += ["rt_gamma_plateau", "rt_stream_probe", "rt_march_probe"]


def rt_stream_probe(ins, outs, blocks: int, reps: int, stream: int | None = None):
    """ins, outs: lists of equal-size float32 device tensors.  Returns
    (code, average ms per launch)."""
    L = lib()
    vp = ctypes.c_void_p
    L.rt_stream_probe.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp),
                                  ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp]
    L.rt_stream_probe.restype = ctypes.c_int
    a = (vp * len(ins))(*[t.data_ptr() for t in ins])
    b = (vp * len(outs))(*[t.data_ptr() for t in outs])
    ms = ctypes.c_double()
    rc = L.rt_stream_probe(a, len(ins), b, len(outs), int(ins[0].numel()), int(blocks),
                           int(reps), ctypes.byref(ms), vp(stream or 0))
    return rc, ms.value


def rt_march_probe(ins, outs, shape, reps: int, stream: int | None = None):
    """ins: 7, outs: 6 float32 device tensors of nz*ny*nx elements; shape =
    (nz, ny, nx).  Returns (code, average ms per launch)."""
    L = lib()
    vp = ctypes.c_void_p
    L.rt_march_probe.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_double), vp]
    L.rt_march_probe.restype = ctypes.c_int
    nz, ny, nx = (int(v) for v in shape)
    if len(ins) != 7 or len(outs) != 6 or any(t.numel() != nx * ny * nz for t in ins + outs):
        return RT_E_ARG, 0.0
    a = (vp * 7)(*[t.data_ptr() for t in ins])
    b = (vp * 6)(*[t.data_ptr() for t in outs])
    ms = ctypes.c_double()
    rc = L.rt_march_probe(a, b, nx, ny, nz, int(reps), ctypes.byref(ms), vp(stream or 0))
    return rc, ms.value


def rt_gamma_plateau(ctx, nH_max: float):
    """Returns (code, gamma0, ncells)."""
    L = lib()
    L.rt_gamma_plateau.argtypes = [ctypes.c_void_p, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
    L.rt_gamma_plateau.restype = ctypes.c_int
    g = ctypes.c_double()
    n = ctypes.c_int64()
    rc = L.rt_gamma_plateau(ctx, float(nH_max), ctypes.byref(g), ctypes.byref(n))
    return rc, g.value, n.value
