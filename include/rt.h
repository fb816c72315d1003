/*
 * rt.h -- C ABI of librt_m1.so: one explicit M1 radiative-transfer step
 * fused with hydrogen photo-chemistry, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Aubert & Teyssier (2010), "Reionization simulations powered by
 * GPUs I".  Sec. 2.2 gives the two-moment equations for the photon number
 * density N and flux F with the M1 closure, their explicit integration under
 * dt < dx/c with Lax-Friedrichs intercell fluxes, and the hydrogen chemistry
 * and cooling sub-cycled within a step; Sec. 2.3 gives the nearest-grid-point
 * point sources; Appendix A gives the explicit update from time p to p+1
 * followed by the per-cell operator Phi (chemistry, temperature, absorption).
 *
 * Conventions shared by every entry point
 *   - Every function returns RT_OK (0) or a negative RT_E_* code; nothing
 *     throws across the ABI.  rt_strerror() names a code.
 *   - Fields are FP32, structure-of-arrays, row-major with x fastest: the
 *     cell (i, j, k) lives at index (k * ny + j) * nx + i.  nx*ny*nz must be
 *     below 2^32.
 *   - Units are CGS: N [photons cm^-3], F [photons cm^-2 s^-1], xHI the
 *     neutral hydrogen fraction, T [K], nH [cm^-3] (must be > 0), dx [cm],
 *     dt [s], source rates [photons s^-1].
 *   - A context serves one grid on one HIP stream and is not re-entrant:
 *     calls on one context must not overlap.  Device work is enqueued on
 *     the context's stream; only rt_reduce, rt_state, rt_profile_read and
 *     rt_destroy wait for it.
 */
#ifndef RT_M1_H
#define RT_M1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define RT_OK 0
#define RT_E_ARG (-1)       /* invalid argument (sizes, enums, ranges)      */
#define RT_E_CFL (-2)       /* dt above the light-crossing bound dx/(3c)    */
#define RT_E_STATE (-3)     /* call out of order / null context             */
#define RT_E_HIP (-4)       /* HIP runtime failure                          */
#define RT_E_NONFINITE (-5) /* a step produced a NaN or Inf (rt_reduce)     */
#define RT_E_NOMEM (-6)     /* allocation of library scratch failed         */

/* ---- boundary conditions, per face in the order -x,+x,-y,+y,-z,+z ------ */
#define RT_BC_PERIODIC 0 /* wrap (both faces of an axis must be periodic)  */
#define RT_BC_OUTFLOW 1  /* zero-gradient copy of the edge cell            */
#define RT_BC_REFLECT 2  /* copy with the face-normal flux negated         */

/* ---- chemistry modes --------------------------------------------------- */
#define RT_CHEM_FULL 0       /* photoionisation, recombination, energy     */
#define RT_CHEM_ISOTHERMAL 1 /* as FULL with T held fixed                  */
#define RT_CHEM_OFF 2        /* transport and sources only                 */
#define RT_CHEM_FROZEN 3     /* absorption by the fixed neutral density    */

/* ---- precision of the chemistry ---------------------------------------- */
#define RT_PREC_FP32 0  /* every cell in FP32                               */
#define RT_PREC_MIXED 1 /* FP64 for cells with xHI < xhi_fp64_thr at step
                           start, FP32 elsewhere                            */

/* ---- chemistry sub-cycling --------------------------------------------- */
#define RT_SUB_FIXED 0    /* nsub equal sub-cycles per step                 */
#define RT_SUB_ADAPTIVE 1 /* h = min(rest, sub_eps * t_chem), at most nsub  */

/* ---- field selectors for rt_state -------------------------------------- */
#define RT_FIELD_N 0
#define RT_FIELD_FX 1
#define RT_FIELD_FY 2
#define RT_FIELD_FZ 3
#define RT_FIELD_XHI 4
#define RT_FIELD_T 5
#define RT_FIELD_NH 6

typedef struct rt_ctx rt_ctx;

/* Device pointers owned by the caller (e.g. torch tensors) and borrowed by
 * the context until rt_destroy.  N and F are double-buffered: index 0 holds
 * the initial state; every step reads buffer `cur` and writes buffer
 * 1 - cur (rt_current reports `cur`).  xHI and T are updated in place; nH is
 * read only.  All buffers hold nx*ny*nz floats, 256-byte alignment or
 * better recommended, and must not alias one another. */
typedef struct {
    float *N[2];
    float *Fx[2];
    float *Fy[2];
    float *Fz[2];
    float *xHI;
    float *T;
    const float *nH;
} rt_fields;

/* Physical and numerical parameters.  sigma_n, sigma_e and egamma_eV are the
 * gray single-group constants of Sec. 2.2 (2.93e-18 cm^2, 2.49e-18 cm^2,
 * 20.27 eV); c_cms the speed of light used by the transport; T_floor [K]
 * bounds T from below; sub_eps the adaptive sub-cycle fraction;
 * xhi_fp64_thr the neutral fraction below which RT_PREC_MIXED switches a
 * cell's chemistry to FP64. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t bc[6];
    int32_t chem;
    int32_t prec;
    int32_t sub;
    int32_t reserved; /* must be 0 */
    double dx_cm;
    double c_cms;
    double sigma_n;
    double sigma_e;
    double egamma_eV;
    double T_floor;
    double sub_eps;
    double xhi_fp64_thr;
} rt_params;

/* Global averages (Sec. 3.1 and 3.2 use the volume- and mass-weighted
 * neutral fractions and the volume-averaged photoionisation rate) and the
 * photon budget.  Sums are accumulated in FP64.  Photon counts are absolute
 * numbers of photons: photons_initial + photons_emitted + photons_floor =
 * photons_stored + photons_absorbed + photons_escaped up to rounding. */
typedef struct {
    double t;                /* simulated time since rt_init [s]            */
    double xhi_vol;          /* <xHI> over cells                            */
    double xhi_mass;         /* sum nH xHI / sum nH                         */
    double gamma_vol;        /* <c sigma_n N> over cells [1/s]              */
    double photons_initial;  /* sum N dx^3 at rt_init                       */
    double photons_emitted;  /* sum over steps of dt * sum of source rates  */
    double photons_stored;   /* sum N dx^3 now                              */
    double photons_absorbed; /* photoionisations, cumulative                */
    double photons_escaped;  /* net outflow through outflow faces           */
    double photons_floor;    /* added by the N >= 0 guard, cumulative       */
    int64_t steps;           /* rt_step calls since rt_init                 */
    int64_t n_nonfinite;     /* cells with a non-finite result, cumulative  */
    int64_t n_fp64;          /* cell-steps whose chemistry ran in FP64      */
    int64_t n_fallback;      /* surrogate cell-steps sent to the exact path */
    int64_t subcycle_hist[8]; /* cell-steps by sub-cycle count: 1, 2-3,
                                 4-7, 8-15, 16-31, 32-63, 64-127, >=128     */
} rt_reductions;

/* Create a context for the grid described by `params` over the caller's
 * `fields`, enqueuing work on `hip_stream` (a hipStream_t; NULL = the null
 * stream).  Validates every parameter on the host before any HIP call
 * (RT_E_ARG), then allocates the library's own small device scratch (block
 * partial sums, source lists), and sums the initial state.  On success *out
 * owns that scratch until rt_destroy.  Sec. 2.2 (constants), Appendix A
 * (the host only drives the device). */
int rt_init(const rt_params *params, const rt_fields *fields, void *hip_stream,
            rt_ctx **out);

/* Replace the point sources (Sec. 2.3): n sources at host arrays ijk
 * (int32, 3n, as i j k = x y z cell indices) with effective rates ndot
 * (double, n, photons/s, escape fraction and boost already folded in).
 * Sources are projected by nearest grid point; each cell emits
 * S = sum ndot / dx^3.  n = 0 removes all sources.  Indices out of range or
 * negative / non-finite rates give RT_E_ARG and leave the previous set in
 * place.  Waits for the stream before replacing the device copy. */
int rt_inject_sources(rt_ctx *ctx, int64_t n, const int32_t *ijk,
                      const double *ndot);

/* Advance one radiative-transfer step of length dt (Appendix A): the
 * unsplit explicit update of (N, F) with Lax-Friedrichs fluxes of the M1
 * system plus dt*S, then Phi per cell -- nsub chemistry sub-cycles (fixed
 * mode) or at most nsub (adaptive mode) -- and the global sums, all in one
 * fused kernel followed by a one-block finalisation.  dt must satisfy
 * dt <= dx/(3c) (the CFL bound of Sec. 2.2 for the 3-D unsplit update;
 * RT_E_CFL otherwise); 1 <= nsub <= 4096.  Asynchronous. */
int rt_step(rt_ctx *ctx, double dt, int32_t nsub);

/* Wait for the stream and report the sums of the last step (or of the
 * initial state before any step) and the cumulative tallies.  Returns
 * RT_E_NONFINITE (with *out filled) if any step produced a non-finite
 * value. */
int rt_reduce(rt_ctx *ctx, rt_reductions *out);

/* Copy field `field` (RT_FIELD_*) of the current state into dst (nx*ny*nz
 * floats; device memory if dst_on_device != 0, else host memory) and wait
 * for the copy. */
int rt_state(rt_ctx *ctx, int32_t field, void *dst, int32_t dst_on_device);

/* Index (0 or 1) of the N/F buffer that holds the current state. */
int rt_current(rt_ctx *ctx, int32_t *index);

/* Start (enable != 0) or stop timing the fused step kernel with HIP events
 * on the context's stream; starting resets the totals. */
int rt_profile(rt_ctx *ctx, int32_t enable);

/* Wait for the stream; total milliseconds and launch count of the fused
 * step kernel since profiling was started. */
int rt_profile_read(rt_ctx *ctx, double *ms_total, int64_t *launches);

/* Release the context and its scratch (never the caller's fields). */
int rt_destroy(rt_ctx *ctx);

/* Static string naming a return code. */
const char *rt_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* RT_M1_H */
