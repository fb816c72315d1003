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
#define RT_E_SCRATCH (-7)   /* request larger than the fixed scratch of an
                               allocation-free entry point                 */

/* ---- boundary conditions, per face in the order -x,+x,-y,+y,-z,+z ------ */
#define RT_BC_PERIODIC 0 /* wrap (both faces of an axis must be periodic)  */
#define RT_BC_OUTFLOW 1  /* zero-gradient copy of the edge cell            */
#define RT_BC_REFLECT 2  /* copy with the face-normal flux negated         */

/* ---- chemistry modes --------------------------------------------------- */
#define RT_CHEM_FULL 0       /* photoionisation, recombination, energy     */
#define RT_CHEM_ISOTHERMAL 1 /* as FULL with T held fixed                  */
#define RT_CHEM_OFF 2        /* transport and sources only                 */
#define RT_CHEM_FROZEN 3     /* absorption by the fixed neutral density    */

/* ---- intercell flux of the transport (Sec. 2.2) ------------------------- */
#define RT_FLUX_LF 0  /* Lax-Friedrichs: signal speeds -c, +c (the paper's) */
#define RT_FLUX_HLL 1 /* HLL: signal speeds c times the extreme eigenvalues
                         of the M1 flux Jacobian on the two sides of a face */

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
 * better recommended, and must not alias one another.
 *
 * Placement: a step streams all eleven buffers at the same cell index at
 * once, so their relative offsets decide how the traffic spreads over the
 * HBM channels.  Separate allocations of equal power-of-two-ish sizes tend
 * to sit at large aligned distances from one another (on one MI355X the
 * 1024^3 LF step took 12.2 ms on such fields); carving them from one
 * allocation at a stride of the 256-byte-rounded field size plus 256 bytes,
 * so that buffer k starts k * 256 bytes off that alignment, took 10.7 ms
 * (the Python binding's RTGrid lays them out so). */
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
 * cell's chemistry to FP64.
 *
 * Subgrid clumping (Sec. 3.2.1, clumping factors of the cell-averaged
 * chemistry equation), active when clump = 1, with nH in cm^-3:
 *   C_R(nH) = max(1, clump_cr_norm * nH^clump_cr_exp)  recombination factor,
 *   C_I(nH) = clump_ci_norm * nH^clump_ci_exp           photoionisation factor.
 * C_I multiplies the photoionisation rate (and so the photons absorbed);
 * C_R multiplies the terms in ne*nHII (case-B recombination, its cooling,
 * bremsstrahlung).  clump = 0 leaves the operator unclumped and the four
 * doubles unused.  The paper fits C_R ~ nH^0.7 and C_I ~ nH^0.1-0.2 (or
 * C_I = 1 with C_R ~ nH^2.5); it shows the normalisations only in figures. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t bc[6];
    int32_t chem;
    int32_t prec;
    int32_t sub;
    int32_t clump;    /* 0 off, 1 power-law clumping factors */
    int32_t flux;     /* RT_FLUX_LF or RT_FLUX_HLL */
    double dx_cm;
    double c_cms;
    double sigma_n;
    double sigma_e;
    double egamma_eV;
    double T_floor;
    double sub_eps;
    double xhi_fp64_thr;
    double clump_cr_norm, clump_cr_exp; /* C_R law (clump = 1) */
    double clump_ci_norm, clump_ci_exp; /* C_I law (clump = 1) */
} rt_params;

/* Global averages (Sec. 3.1.1-3.1.3 use the volume- and mass-weighted
 * neutral fractions and the volume-averaged photoionisation rate) and the
 * photon budget.  Sums are accumulated in FP64.  Photon counts are absolute
 * numbers of photons: photons_initial + photons_emitted + photons_floor =
 * photons_stored + photons_absorbed + photons_escaped + photons_diluted up
 * to rounding. */
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
    int64_t n_fallback;      /* learned-chemistry cell-steps whose prediction
                                was rejected (the exact operator took them) */
    int64_t subcycle_hist[8]; /* cell-steps by sub-cycle count: 1, 2-3,
                                 4-7, 8-15, 16-31, 32-63, 64-127, >=128     */
    double tau_e;            /* Thomson depth c sigma_T sum_steps <nH (1 - xHI)> dt,
                                with the state at the end of each step (Sec. 3.1.4) */
    int64_t n_learned;       /* learned-chemistry cell-steps that kept the
                                network's prediction, cumulative */
    int64_t n_fallback_range; /* of n_fallback, the cell-steps rejected
                                 because an input left the training range */
    double photons_diluted;  /* removed by the expansion's dilution
                                (rt_set_expansion), cumulative */
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

/* Sources from the stellar particles of a snapshot (Sec. 2.3), for the
 * interval [t_p, t_next] (seconds, 0 < t_p < t_next; t is the age of the
 * Universe); replaces the context's source set like rt_inject_sources.
 * Device arrays of n particles: pos (3n doubles, x y z in cm, wrapped into
 * the periodic box of nx*dx by ny*dx by nz*dx), age_next (age at t_next, s),
 * lifetime (ionising lifetime L > 0, s), q_per_baryon (ionising photons per
 * stellar baryon over L, >= 0), mass_g (>= 0, g).  A particle emits
 * Ndot = Q m / m_b / L (m_b = 1.67262192e-24 g) while its age lies in
 * [0, L]; over the interval it is given the rate Ndot * overlap / Delta
 * (Delta = t_next - t_p; overlap = the time its emitting ages share with
 * [age_next - Delta, age_next]: the photons it emits within the interval,
 * spread evenly over it), times f_esc (in [0, 1]) and the boost factor
 * B = max(1, a_b exp(k_b / t_mid)) at the interval's middle (a_b >= 0,
 * k_b >= 0 in s).  Each particle goes to the cell holding it (nearest grid
 * point), duplicate cells summed in particle order.  *n_active (host, may be
 * NULL) receives the number of emitting particles.  RT_E_ARG for invalid
 * scalars or particles (non-finite values, L <= 0, negative Q or m), leaving
 * the previous source set.  Waits for the stream. */
int rt_sources_from_particles(rt_ctx *ctx, int64_t n, const double *pos,
                              const double *age_next, const double *lifetime,
                              const double *q_per_baryon, const double *mass_g, double t_p,
                              double t_next, double f_esc, double a_b, double k_b,
                              int64_t *n_active);

/* Advance one radiative-transfer step of length dt (Appendix A): the
 * unsplit explicit update of (N, F) with the intercell fluxes of
 * rt_params.flux (Lax-Friedrichs or HLL) of the M1 system plus dt*S, then
 * Phi per cell -- nsub chemistry sub-cycles (fixed mode) or at most nsub
 * (adaptive mode) -- and the global sums.  One fused kernel sweeps the
 * grid; the cells whose Phi is costly -- in mixed precision those below
 * xhi_fp64_thr (FP64 chemistry), in the adaptive and learned forms those
 * that need more than one sub-cycle -- are left to a second kernel that
 * processes them in dense wavefronts; a last one finalises the sums.  dt
 * must satisfy dt <= dx/(3c) (the CFL bound of Sec. 2.2 for the 3-D unsplit
 * update; RT_E_CFL otherwise); 1 <= nsub <= 4096.  Asynchronous, except
 * that a step whose tiling has no source lists yet first bins the point
 * sources for it (waiting for the stream once).  RT_E_STATE also if the
 * context's partial-sum buffer could not hold the launch (an internal
 * check; nothing is launched then). */
int rt_step(rt_ctx *ctx, double dt, int32_t nsub);

/* Expansion of the medium for the steps that follow (the runs of Sec. 2.1-
 * 2.3 span some 800 Myr of cosmic time on comoving boxes; the moment
 * equations of Sec. 2.2 carry no expansion terms).  hubble = H = (da/dt)/a
 * [1/s], in the proper frame, held constant over each step: after the
 * transport update of a step, N and F are multiplied by exp(-3 H dt) (the
 * photon number density and number flux dilute alike, so the reduced flux
 * and the M1 closure are unchanged) and, with RT_CHEM_FULL, T by
 * exp(-2 H dt) (adiabatic cooling of a monatomic gas); then the chemistry.
 * The photons removed accumulate in rt_reductions.photons_diluted.  nH and
 * the cell size are not changed: the caller writes each snapshot's density
 * into the nH field and creates the context with the interval's proper cell
 * size.  0 (the default) is a static medium, bit-identical to a context that
 * never called this.
 * RT_E_ARG unless 0 <= hubble < infinity, RT_E_STATE for a NULL ctx. */
int rt_set_expansion(rt_ctx *ctx, double hubble);

/* Switch the learned chemistry on (theta != NULL) or off (theta == NULL).
 * Not part of the paper's method.  theta: device, RT_MLP_NPARAM FP32 network
 * parameters (copied into the context's own packed bf16 operands, so the
 * caller may free it afterwards).  The network maps the standardised log10
 * features (nH, xHI, T, N, dt; xHI and N floored at 1e-30) to the
 * standardised u = asinh(d / 1e-3) of the changes d = log10(xHI'/xHI) and
 * d = log10(T'/T) over dt (linear for small changes, logarithmic for
 * large ones; decoded as d = 1e-3 sinh u).  norm: host
 * float[24] = mu_in[5], sd_in[5], mu_out[2], sd_out[2] (the two
 * standardisations) and in_min[5], in_max[5] (the training range of the raw
 * log10 features).  With it on and chem == RT_CHEM_FULL, rt_step asks the
 * network, on the matrix cores, for the cells whose chemistry is costly:
 * those that are not dark (photons after transport, or xHI < 1) and whose
 * adaptive operator would take more than one sub-cycle (sub_eps times the
 * chemistry time scale at the transported state below dt; sub_eps = 0 asks
 * it for every such cell), plus, in mixed precision, the cells below
 * xhi_fp64_thr.  For each it derives the absorbed photons from the predicted
 * (xHI', T') (net ionisations + recombinations - collisional ionisations
 * over dt at that state) so the photon budget stays exact, and runs the
 * exact Phi of the context's mode instead for any cell whose inputs leave
 * the training range, whose prediction leaves the physical bounds, or whose
 * backward-Euler residuals over dt (photoionisation, energy) exceed
 * residual_tol (rt_reductions.n_fallback; n_learned counts the accepted
 * cells).  The other cells take the exact operator.  RT_E_ARG for
 * non-positive scales or tol, an inverted training range or sub_eps outside
 * [0, 1]. */
int rt_set_surrogate(rt_ctx *ctx, const float *theta, const float *norm, double residual_tol);

/* Wait for the stream and report the sums of the last step (or of the
 * initial state before any step) and the cumulative tallies: the volume-
 * and mass-weighted neutral fractions and the volume-averaged
 * photoionisation rate whose histories Sec. 3.1.1-3.1.3 follow, the photon
 * budget, and the Thomson depth of Sec. 3.1.4.  Returns RT_E_NONFINITE
 * (with *out filled) if any step produced a non-finite value. */
int rt_reduce(rt_ctx *ctx, rt_reductions *out);

/* Quantities binned by rt_histogram against the cell density. */
#define RT_HQ_XHI 0   /* neutral fraction xHI                     */
#define RT_HQ_GAMMA 1 /* photoionisation rate c sigma_n N [1/s]   */
#define RT_HIST_MAX_BINS 8192 /* nbx * nby                         */

/* Distribution of the current cells over density and a quantity (Sec. 3.1.5
 * studies xHI(nH) and J21(nH) this way, with the mean per density bin).
 * Bins: nbx bins in nH between 10^lox and 10^hix and nby bins in q between
 * 10^loy and 10^hiy, uniform in log10, with FP64 edges e_k = pow(10, lo +
 * k w), w = (hi - lo) / nb; a value falls in the largest k < nb with
 * e_k <= value, values below e_0 (zero included) in bin 0.  q = xHI, or
 * (c_cms * sigma_n) * N evaluated in FP64 for RT_HQ_GAMMA.
 * counts (host, nbx * nby int64, row ix: counts[ix * nby + iy]) receives
 * the exact cell counts; sum_q (host, nbx doubles) the sum of q over the
 * cells of each density bin: xHI (resp. N) is summed exactly in fixed point,
 * independent of the order of the additions, rounded to FP64 (a few ulp)
 * and, for RT_HQ_GAMMA, multiplied by c_cms * sigma_n in FP64, so the same
 * state gives the same sums bit for bit; a negative or non-finite value
 * makes its bin's sum NaN.  Both are overwritten.  1 <= nbx, nby <= 256, nbx * nby <= RT_HIST_MAX_BINS,
 * lo < hi, |lo|, |hi| <= 300, else RT_E_ARG.  Waits for the stream. */
int rt_histogram(rt_ctx *ctx, int32_t quantity, int32_t nbx, double lox, double hix,
                 int32_t nby, double loy, double hiy, int64_t *counts, double *sum_q);

/* Self-shielding models of the photoionisation rate against density
 * (Sec. 3.1.5 fits the intensity of its runs by a plateau J0 with an
 * exponential cutoff; with the gray constants the rate is proportional to the
 * intensity, so the models apply to Gamma). */
#define RT_JMODEL_UNIFORM 0 /* Gamma(nH) = gamma0                    (J0) */
#define RT_JMODEL_EXP1 1    /* Gamma(nH) = gamma0 exp(-nH / n_star)  (J1) */
#define RT_JMODEL_EXP4 2    /* Gamma(nH) = gamma0 exp(-(nH/n_star)^4) (J4) */

/* Equilibrium neutral fraction under a model (Sec. 3.1.5 compares the mean
 * neutral fraction per density bin with it; clumped as in Sec. 3.2.1): per
 * element, Gamma = model(nH[i]) and xhi[i] = the root y in [0, 1] of
 *   C_R alpha_B(T) nH (1 - y)^2 = C_I Gamma y + beta(T) nH (1 - y) y,
 * the fixed point of the chemistry operator at fixed T[i] and Gamma (case-B
 * recombination against photo- and collisional ionisation; the same rate
 * fits as rt_step).  nH, T, xhi: device arrays of n FP64 values,
 * caller-owned; an element with nH <= 0 or non-finite, or T outside
 * [1, 1e9] K, gives NaN.  params: host; only the clumping fields are read
 * (C_R = C_I = 1 when clump = 0), validated as by rt_init.  gamma0 >= 0 and
 * finite; n_star > 0 and finite unless model = RT_JMODEL_UNIFORM;
 * 0 <= n < 2^31 (RT_E_ARG otherwise).  Asynchronous on hip_stream (NULL:
 * the null stream). */
int rt_equilibrium_xhi(const rt_params *params, int32_t model, double gamma0, double n_star,
                       int64_t n, const double *nH, const double *T, double *xhi,
                       void *hip_stream);

/* Plateau of the photoionisation rate (Sec. 3.1.5: at low density the
 * intensity of a run is nearly constant, and its mean there is taken as the
 * J0 of the self-shielding models): *gamma0 = the mean of c_cms * sigma_n * N
 * over the cells of the current state with nH < nH_max [cm^-3], in FP64 and
 * in a fixed summation order; *ncells (may be NULL) receives how many cells
 * that is.  RT_E_ARG for nH_max not positive and finite, or when no cell lies
 * below it (*ncells = 0 then).  Waits for the stream. */
int rt_gamma_plateau(rt_ctx *ctx, double nH_max, double *gamma0, int64_t *ncells);

/* Copy field `field` (RT_FIELD_*) of the current state into dst (nx*ny*nz
 * floats; device memory if dst_on_device != 0, else host memory) and wait
 * for the copy: the output step of Appendix A, where the host reads the
 * fields back from the device (the paper every few thousand steps). */
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

/* ---- exact chemistry on a batch of independent cells ------------------- */

/* Apply the per-cell operator Phi (Appendix A; the sub-cycled hydrogen
 * chemistry and cooling of Sec. 2.2) to n independent cells, in place, on
 * `hip_stream`, exactly as rt_step applies it after transport: nH, N, xHI,
 * T and dt are device arrays of n floats (dt per cell, seconds); N, xHI and
 * T are updated; ncycles (device int32[n], may be NULL) receives the number
 * of sub-cycles each cell took.  Only the chemistry fields of `params` are
 * read (chem, prec, sub, sub_eps, T_floor, xhi_fp64_thr, c_cms, sigma_n,
 * sigma_e, egamma_eV); grid sizes and boundaries are ignored.  Used to
 * produce training pairs for the surrogate.  Asynchronous. */
int rt_chem_apply(const rt_params *params, int64_t n, const float *nH, float *N,
                  float *xHI, float *T, const float *dt, int32_t nsub, int32_t *ncycles,
                  void *hip_stream);

/* ---- the chemistry-surrogate network (bf16 matrix cores) --------------- */
/* Not part of the paper's method: an optional learned replacement for Phi.
 * Network 5 -> 64 -> 64 -> 64 -> 2, SiLU hidden units.  theta is a device
 * array of RT_MLP_NPARAM FP32 values in the order W1 (64x5), b1, W2 (64x64),
 * b2, W3 (64x64), b3, W4 (2x64), b4, each W row-major (out, in).  Products
 * run on bf16 operands rounded from theta and X with FP32 accumulation. */
#define RT_MLP_NPARAM 8834

typedef struct rt_mlp rt_mlp;

/* Workspace for forward/gradient calls on `hip_stream`; grad_blocks (1 ..
 * 65536) sets how many blocks of four wavefronts share a gradient evaluation
 * (each keeps an FP32 gradient partial: grad_blocks * 8834 floats; one
 * block per compute unit runs at a time, so 256 fill an MI355X). */
int rt_mlp_create(int32_t grad_blocks, void *hip_stream, rt_mlp **out);

/* Y (device, B x 2) = network(X (device, B x 5, standardised inputs)). */
int rt_mlp_forward(rt_mlp *m, const float *theta, const float *X, int64_t B, float *Y);

/* Gradient of L = 1/(2B) sum over samples and outputs of (y - Y)^2 with
 * respect to theta into grad (device, 8834 FP32); loss_dev (device double,
 * may be NULL) receives L.  Deterministic (fixed-order reduction). */
int rt_mlp_grad(rt_mlp *m, const float *theta, const float *X, const float *Y, int64_t B,
                float *grad, double *loss_dev);

/* One Adam step (Kingma & Ba 2015, bias-corrected, step >= 1) on the FP32
 * master theta with moment buffers mom1, mom2 (device, 8834 each). */
int rt_mlp_adam(rt_mlp *m, float *theta, float *mom1, float *mom2, const float *grad,
                int64_t step, double lr, double beta1, double beta2, double eps);

int rt_mlp_destroy(rt_mlp *m);

/* Training pairs for the surrogate, on `hip_stream`: for n independent cells
 * (device arrays of n floats nH, N, xHI, T, dt; not modified) the features
 * X (device, n x 5: log10 of nH, max(xHI, 1e-30), T, max(N, 1e-30), dt) and,
 * with the exact operator Phi applied to a copy of each cell exactly as
 * rt_chem_apply applies it (the chemistry fields of params, nsub as there),
 * the targets U (device, n x 2: u = asinh(d / 1e-3) of the changes
 * d = log10(xHI'/xHI), log10(T'/T), xHI floored likewise), the end values
 * Yend (device, n x 2: log10 xHI', log10 T') and the sub-cycles each cell
 * took (ncycles, device int32[n]).  Logarithms and the encoding in FP64.
 * Any of X, U, Yend, ncycles may be NULL (not all); with U, Yend and ncycles
 * NULL the chemistry is skipped.  RT_E_ARG as rt_chem_apply.  Asynchronous. */
int rt_mlp_pairs(const rt_params *params, int64_t n, const float *nH, const float *N,
                 const float *xHI, const float *T, const float *dt, int32_t nsub, float *X,
                 float *U, float *Yend, int32_t *ncycles, void *hip_stream);

/* Column standardisation of A (device, n x d FP32, 1 <= d <= 8): stats
 * (device, 4 d doubles) receives the column means, standard deviations
 * (sqrt of the sum of squared deviations / (n - 1), at least 1e-6; 1 for
 * n = 1), minima and maxima, all summed in FP64 in a fixed order; out
 * (device, n x d, may be A) receives (A - mean) / sd.  Uses the workspace's
 * partial-sum buffers; asynchronous on its stream. */
int rt_mlp_standardize(rt_mlp *m, const float *A, int64_t n, int32_t d, float *out,
                       double *stats);

/* Options of rt_mlp_train. */
typedef struct {
    int64_t batch;       /* samples per step, >= 1                            */
    int64_t total_steps; /* length of the learning-rate schedule, >= 1         */
    double lr;           /* peak learning rate, > 0                            */
    double warmup;       /* fraction of total_steps with a linear rise, [0, 1) */
    double lr_floor;     /* added to the cosine decay, >= 0                    */
    double clip;         /* global gradient-norm bound; <= 0: no clipping      */
    double beta1, beta2, eps; /* Adam                                          */
    uint64_t seed;       /* batch sampling                                     */
} rt_mlp_train_opts;

/* Steps step0 + 1 .. step0 + nsteps (step0 + nsteps <= total_steps) of
 * minibatch training of the network on the standardised pairs X (device,
 * n x 5) -> Y (device, n x 2), 1 <= n < 2^31: each step draws its batch on
 * the device (sample i is row floor(h n / 2^32), h the upper 32 bits of
 * SplitMix64 (Steele, Lea & Flood 2014) at k + i, k = SplitMix64(seed XOR
 * (step * 0xD1B54A32D192ED03)); rows may repeat), takes the gradient of
 * rt_mlp_grad on it, rescales the gradient to global norm clip when above
 * it (norm summed in FP64, fixed order), and makes the Adam step of
 * rt_mlp_adam with the learning rate lr s / n_w over the first
 * n_w = max(1, floor(warmup total_steps)) steps s and lr (1 + cos(pi (s -
 * n_w) / max(total_steps - n_w, 1))) / 2 + lr_floor after them.  theta,
 * mom1, mom2 as rt_mlp_adam (mom1, mom2 zero before the first step);
 * loss_dev (device double, may be NULL) receives the last step's batch
 * loss.  A run split into several calls equals one call.  Asynchronous. */
int rt_mlp_train(rt_mlp *m, float *theta, float *mom1, float *mom2, const float *X,
                 const float *Y, int64_t n, const rt_mlp_train_opts *opts, int64_t step0,
                 int64_t nsteps, double *loss_dev);

/* The trained network on raw features X (device, n x 5, as rt_mlp_pairs
 * writes them): standardised with norm (host, 14 floats: mu_in[5] sd_in[5]
 * mu_out[2] sd_out[2], sd > 0), evaluated, destandardised to u and decoded
 * to the end values Y (device, n x 2, may be NULL): log10 xHI' = X[1] +
 * 1e-3 sinh(u0), log10 T' = X[2] + 1e-3 sinh(u1).  With targets U (device,
 * n x 2, encoded as rt_mlp_pairs writes them) loss_dev (device double)
 * receives the mean over samples and both outputs of the squared
 * standardised error (the training loss); loss_dev NULL skips it.
 * Asynchronous. */
int rt_mlp_predict(rt_mlp *m, const float *theta, const float *norm, const float *X, int64_t n,
                   float *Y, const float *U, double *loss_dev);

/* rt_mlp_grad without a workspace object, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight training loops,
 * harnesses that forbid allocation.  It allocates nothing: the packed
 * operands and the per-block gradient partials live in one fixed library
 * array per device (RT_MLP_NOALLOC_BYTES, about 9 MB, reserved when the
 * library is loaded and held until the process ends).  grad_blocks plays
 * the role of rt_mlp_create's: 1 .. RT_MLP_NOALLOC_BLOCKS, RT_E_SCRATCH
 * above (RT_E_ARG below 1 or for the other arguments, as rt_mlp_grad).
 * The first call on a device looks up the array's address on that device
 * (the device of hip_stream, or the current device for the null stream);
 * make it before a graph capture begins.  With the same grad_blocks the
 * result equals rt_mlp_grad's bit for bit (the same kernels and summation
 * order).  Every call on a device uses the same array: calls that may
 * overlap on one device (unordered streams, concurrent host threads) race;
 * calls ordered on one stream do not.  Asynchronous on hip_stream. */
#define RT_MLP_NOALLOC_BLOCKS 256
#define RT_MLP_NOALLOC_BYTES (256 * 8834 * 4 + 2048 + 40960)
int rt_mlp_grad_noalloc(int32_t grad_blocks, const float *theta, const float *X,
                        const float *Y, int64_t B, float *grad, double *loss_dev,
                        void *hip_stream);

/* ---- measurement utility (not part of the method) --------------------- */

/* The HBM bandwidth the step's stream mix can reach: a plain grid-stride
 * kernel reads nin (1..16) device arrays in[k] of n floats and writes nout
 * (1..16) arrays out[k] (non-temporal stores, each output depending on every
 * input), `blocks` blocks of 256 threads; one warm-up launch, then reps
 * launches timed with HIP events on hip_stream.  *ms receives the average
 * launch time; (nin + nout) * 4 * n bytes move per launch.  Arrays are
 * caller-owned and must not alias.  Waits for the stream. */
int rt_stream_probe(const float *const *in, int32_t nin, float *const *out, int32_t nout,
                    int64_t n, int32_t blocks, int32_t reps, double *ms, void *hip_stream);

/* The same 7-read / 6-write mix in the LF step kernel's access order: 64 x
 * 16 tiles of 1024 threads, one per block and one block per compute unit
 * (96 KiB of LDS each), march 128 planes in z with the next plane's loads
 * in flight and one barrier per plane, over an nx x ny x nz grid (x
 * fastest; nx a multiple of 64, ny of 16, nz of 128, else RT_E_ARG) of
 * in[0..6] (read) and out[0..5] (written, non-temporal stores); no stencil,
 * halo, sources or chemistry.  One warm-up launch, then reps launches timed
 * with HIP events on hip_stream; *ms receives the average launch time, in
 * which 52 bytes per cell move.  Arrays are caller-owned, nx ny nz floats
 * each, and must not alias.  Waits for the stream. */
int rt_march_probe(const float *const *in, float *const *out, int32_t nx, int32_t ny,
                   int32_t nz, int32_t reps, double *ms, void *hip_stream);

/* Static string naming a return code. */
const char *rt_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* RT_M1_H */
