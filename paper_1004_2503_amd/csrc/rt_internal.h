// rt_internal.h -- declarations shared by the host side of the C ABI and the
// gfx950 kernels of librt_m1.so.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt.h"

namespace rtk {

// Tile of the fused step kernel: one wavefront per x-row of 64 cells, TY
// rows per block (512 threads), the block marching ZC planes along z.
constexpr int TX = 64;
constexpr int TY = 8;
constexpr int NTHREADS = TX * TY;

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
    R_FALLBACK,    // surrogate cells sent to the exact path
    R_HIST0,       // 8 sub-cycle histogram bins
    NRED = R_HIST0 + 8
};

// Layout of the library's accumulator array (doubles, device).
constexpr int ACC_CUR = 0;    // NRED sums of the last step (or initial state)
constexpr int ACC_CUM = 32;   // NRED cumulative sums over steps
constexpr int ACC_SIZE = 64;

struct StepArgs {
    const float *N, *Fx, *Fy, *Fz;   // current buffer
    float *No, *Fxo, *Fyo, *Fzo;     // next buffer
    float *xHI, *T;                  // in place
    const float *nH;
    const int32_t *src_ptr;          // per block [start, end) into src_key/rate
    const int32_t *src_key;          // (z - z0) * NTHREADS + thread index
    const float *src_rate;           // S = ndot / dx^3 [cm^-3 s^-1]
    double *partials;                // nblocks * NRED
    int nx, ny, nz;
    uint32_t plane;                  // nx * ny
    int ntx, nty, nzc, zc, nblocks;
    int bc[6];
    int chem, mixed, adaptive, nsub, any_outflow;
    // FP32 constants
    float c, inv_c, half_c, half_c2, k1, dt, csig, T_h, inv15kB, T_floor,
        sub_eps, xhi_thr;
    // FP64 constants for the FP64 chemistry path and the tallies
    double dt_d, csig_d, T_h_d, T_floor_d, sub_eps_d, vol, esc_scale;
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
hipError_t launch_mlp_pack(const float *theta, __bf16 *pk, hipStream_t s);
hipError_t launch_finalize(const double *partials, int nblocks, double *acc,
                           int mode, hipStream_t s);
hipError_t launch_state_sums(const float *N, const float *xHI, const float *nH,
                             uint32_t ncell, double *partials, int nblocks,
                             hipStream_t s);
int state_sums_blocks(uint32_t ncell);

}  // namespace rtk
