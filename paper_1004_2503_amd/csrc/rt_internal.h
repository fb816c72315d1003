// rt_internal.h -- declarations shared by the host side of the C ABI and the
// gfx950 kernels of librt_m1.so.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt.h"

namespace rtk {

// Tiles of the fused step kernel: one wavefront per x-row of 64 cells, the
// block marching ZC planes along z.  On large grids the plain LF forms use
// TY_LF rows per block (64 TY_LF threads, at most 128 VGPRs each: more rows
// share each halo row); on small grids (too few such tiles to fill the
// chip) they use TY rows (64 TY threads).  The HLL form, which needs more
// registers per thread, uses TY_HLL rows: 768 threads at up to 168 VGPRs,
// three wavefronts per SIMD (two with 64 x 8 tiles at its 187 VGPRs).
#ifndef RT_M1_TY
#define RT_M1_TY 8
#endif
#ifndef RT_M1_TY_LF
#define RT_M1_TY_LF 16
#endif
#ifndef RT_M1_TY_HLL
#define RT_M1_TY_HLL 12
#endif
constexpr int TX = 64;
constexpr int TY = RT_M1_TY;
constexpr int NTHREADS = TX * TY;
constexpr int TY_LF = RT_M1_TY_LF;
constexpr int NTHREADS_LF = TX * TY_LF;
constexpr int TY_HLL = RT_M1_TY_HLL;
constexpr int NTHREADS_HLL = TX * TY_HLL;
constexpr int NTHREADS_MAX = NTHREADS_LF > (NTHREADS > NTHREADS_HLL ? NTHREADS : NTHREADS_HLL)
                                 ? NTHREADS_LF
                                 : (NTHREADS > NTHREADS_HLL ? NTHREADS : NTHREADS_HLL);
constexpr int SRC_LDS = 256;   // sources staged in LDS per refill

// Per-block partial sums written by the step kernel (all FP64).
enum Red : int {
    R_XHI = 0,     // sum xHI
    R_NHXHI,       // sum nH xHI
    R_NH,          // sum nH
    R_N,           // sum N
    R_ABS,         // photons absorbed this step (dx^3 folded in)
    R_ESC,         // photons escaped this step (dt dx^2 folded in)
    R_FLOOR,       // photons added by the N >= 0 guard (dx^3 folded in)
    R_NONFINITE,   // cells with a non-finite result
    R_FP64,        // cells whose chemistry ran in FP64
    R_FALLBACK,    // learned-chemistry cells whose prediction was rejected
    R_LEARNED,     // learned-chemistry cells that kept the prediction
    R_RANGE,       // learned-chemistry cells rejected for inputs outside the
                   // training range (counted in R_FALLBACK too)
    R_DILUTE,      // photons removed by the expansion's dilution (dx^3 folded in)
    R_HIST0,       // 8 sub-cycle histogram bins
    NRED = R_HIST0 + 8
};

// Layout of the library's accumulator array (doubles, device).
constexpr int ACC_CUR = 0;    // NRED sums of the last step (or initial state)
constexpr int ACC_CUM = 32;   // NRED cumulative sums over steps
constexpr int ACC_SIZE = 64;
constexpr int ACC_TAU = 31;   // ACC_CUM + ACC_TAU: Thomson depth (cumulative)
static_assert(NRED <= ACC_TAU && ACC_CUM + ACC_TAU < ACC_SIZE, "accumulator layout");

// Subgrid clumping laws: C = 2^(exp log2 nH + l2n), l2n = log2 norm; C_R is
// bounded below by 1.  on = 0: C_R = C_I = 1.
struct ClumpLaw {
    int on;
    float cr_exp, cr_l2n, ci_exp, ci_l2n;
};
// The same laws for the FP64 chemistry: C = norm nH^exp.
struct ClumpLawD {
    int on;
    double cr_norm, cr_exp, ci_norm, ci_exp;
};

struct StepArgs {
    const float *N, *Fx, *Fy, *Fz;   // current buffer
    float *No, *Fxo, *Fyo, *Fzo;     // next buffer
    float *xHI, *T;                  // in place
    const float *nH;
    const int32_t *src_ptr;          // per block [start, end) into src_key/rate
    const int32_t *src_key;          // (z - z0) * threads per block + thread index
    const float *src_rate;           // S = ndot / dx^3 [cm^-3 s^-1]
    double *partials;                // nblocks * NRED
    float *sink;                     // NTHREADS_MAX floats: stores of lanes off the grid
    int nx, ny, nz;
    uint32_t plane;                  // nx * ny
    int ntx, nty, nzc, zc, nblocks;  // of the tiles of the form that runs
    int bc[6];
    int chem, mixed, adaptive, nsub, any_outflow;
    int hll;                         // 1: HLL fluxes, 0: LF
    int big;                         // 1: 64 x TY_LF tiles (LF forms, large grids)
    // Cells whose chemistry the step leaves to launch_defer_chem are marked
    // in fp64_mask (one bit per cell, one 64-bit word per x-row of a tile:
    // word (z * ny + y) * ntx + tile x): in mixed precision the cells with
    // xHI < xhi_thr (FP64 chemistry), with defer_stiff the cells whose
    // adaptive operator would take more than one sub-cycle (sub_eps times
    // the chemistry time scale below dt).  The deferred kernel runs the
    // learned chemistry on them when surr is set.
    int defer;                       // mask in use (mixed or defer_stiff)
    int defer_stiff;
    int count_hist;                  // sub-cycle histogram counted on the device
    uint64_t *fp64_mask;
    // one bit per group of 64 consecutive mask words that holds a marked
    // cell (set by the step, cleared by the finalisation): the deferred
    // kernels visit only those groups
    uint64_t *group_mask;
    ClumpLaw cl;
    ClumpLawD cld;
    // expansion at rate H over the step: N, F *= dil3 = exp(-3 H dt) after
    // the transport update, T *= dil2 = exp(-2 H dt) under the full
    // chemistry; one_m_dil3 = 1 - dil3 (rounded once, for the tally)
    int expand;
    float dil3, dil2, one_m_dil3;
    // FP32 constants
    float c, inv_c, half_c, half_c2, k1, dt, csig, T_h, inv15kB, T_floor,
        sub_eps, xhi_thr;
    // FP64 constants for the FP64 chemistry path and the tallies
    double dt_d, csig_d, T_h_d, T_floor_d, sub_eps_d, inv15kB_d, vol, esc_scale;
    double c_d;                      // c in FP64 (HLL reduced flux 1 - f^2)
    // learned chemistry (surrogate form): packed bf16 forward operands,
    // biases b1|b2|b3|b4 (194 floats), and mu_in[5] sd_in[5] mu_out[2]
    // sd_out[2] in_min[5] in_max[5]
    const __bf16 *surr_pk;
    const float *surr_bias;
    float surr_norm[24];
    float surr_tol, log10_dt;
    int surr;
};

constexpr int SURR_NBIAS = 194;
constexpr int SURR_NNORM = 24;

hipError_t launch_step(const StepArgs &a, hipStream_t s);
// The chemistry of the cells marked by the step (StepArgs::defer): with the
// learned chemistry on, first the network on them (nb2 blocks, partial rows
// nblocks .. nblocks + nb2 - 1), which leaves only its rejected cells
// marked; then the exact operator on the marked cells (nb2 blocks, the next
// nb2 rows, or from row nblocks without the network).  defer_rows: the
// partial rows the two take.
int defer_chem_blocks(uint64_t nwords);
__host__ __device__ inline uint64_t mask_groups(uint64_t nwords) { return (nwords + 63) / 64; }
// goff: defer_offsets_size(nwords) entries (group and block offsets);
// cells: one entry per cell of the grid (the dense list of marked cells);
// mask2: a second mask of nwords words (the learned form's rejected cells).
size_t defer_offsets_size(uint64_t nwords);
hipError_t launch_defer_chem(const StepArgs &a, uint64_t nwords, int nb2, uint32_t *goff,
                             uint32_t *cells, uint64_t *mask2, hipStream_t s);
inline int defer_rows(const StepArgs &a, int nb2)
{
    return a.defer ? ((a.surr && a.chem == RT_CHEM_FULL) ? 2 * nb2 : nb2) : 0;
}
ClumpLaw make_clump_law(const rt_params &p);
ClumpLawD make_clump_law_d(const rt_params &p);
int inject_host(rt_ctx *c, int64_t n, const int32_t *ijk, const double *ndot);
hipError_t launch_particle_rates(int64_t n, const double *pos, const double *age_next,
                                 const double *lifetime, const double *q, const double *mass,
                                 double delta, double f_esc, double boost, double dx, int nx,
                                 int ny, int nz, int32_t *ijk, double *rate, int32_t *bad,
                                 hipStream_t s);
int check_clump(const rt_params &p);
hipError_t launch_mlp_pack(const float *theta, __bf16 *pk, hipStream_t s);
// mode 0 also adds tau_coef * (nh_sum - sum nH xHI) to acc[ACC_CUM + ACC_TAU].
// More than FIN1_MIN partial rows go through a first level of FIN1_BLOCKS
// blocks whose rows land in scratch (FIN1_BLOCKS * NRED doubles).
constexpr int FIN1_BLOCKS = 256;
constexpr int FIN1_MIN = 4096;
hipError_t launch_finalize(const double *partials, int nblocks, double *scratch, double *acc,
                           int mode, double tau_coef, double nh_sum, hipStream_t s,
                           uint64_t *clear = nullptr, int nclear = 0);
size_t hist_lds_bytes(int nbx, int nby);
// histogram blocks for ncell cells
constexpr int HIST_MAX_BLOCKS = 2048;
int hist_blocks(uint32_t ncell);
// limbs: hist_limb_count(nbx) zeroed 64-bit words (the exact per-density-bin
// sums); sums: nbx doubles
size_t hist_limb_count(int nbx);
hipError_t launch_hist(const float *nH, const float *q, int gamma, double csig, uint32_t ncell,
                       int nbx, int nby, const double *edges, float lox, float inv_wx,
                       float loy, float inv_wy, unsigned long long *counts,
                       unsigned long long *limbs, double *sums, hipStream_t s);
// plateau: part holds 2 plateau_blocks(ncell) doubles; out 2 (sum, count)
int plateau_blocks(uint32_t ncell);
hipError_t launch_plateau(const float *nH, const float *N, uint32_t ncell, double nh_max,
                          double csig, double *part, double *out, hipStream_t s);
hipError_t launch_equilibrium(int64_t n, const double *nH, const double *T, double *xhi,
                              int model, double gamma0, double n_star, const rt_params &p,
                              hipStream_t s);
hipError_t launch_state_sums(const float *N, const float *xHI, const float *nH,
                             uint32_t ncell, double *partials, int nblocks,
                             hipStream_t s);
int state_sums_blocks(uint32_t ncell);

}  // namespace rtk
