// mlp_device.h -- the chemistry-surrogate network on gfx950 matrix cores.
//
// Network 5 -> 64 -> 64 -> 64 -> 2 with SiLU hidden units, bf16 operands,
// FP32 accumulation, evaluated with v_mfma_f32_32x32x16_bf16 in the
// transposed form  Z (neurons x cells) = W (out x in) . H (in x cells),  so
// that 32 cells form the N dimension of every product.
//
// Lane layouts of the 32x32x16 bf16 product (checked on the device):
//   A (32 x 16): lane l supplies row l%32, k = 8*(l/32) + 0..7;
//   B (16 x 32): lane l supplies column l%32, k = 8*(l/32) + 0..7;
//   D (32 x 32): lane l holds column l%32, rows 8*(r/4) + 4*(l/32) + r%4
//                for r = 0..15.
// A layer's D tiles therefore hold, in lane l, the cell l%32 and 16 of the
// neurons per 32-neuron tile.  Those registers are fed unchanged to the next
// product as its B operand: K-chunk kc (16 inputs) takes registers
// 8*(kc%2) .. +7 of tile kc/2, i.e. input neuron perm_in(kc, l/32, s); the
// weight operand is packed with the same permutation of its input index, so
// no data moves between lanes between layers.
//
// Parameters: one FP32 vector of 8834 values in the order W1 (64x5), b1,
// W2 (64x64), b2, W3 (64x64), b3, W4 (2x64), b4, each W row-major (out, in).
#pragma once

#include "rt_device.h"

namespace rtk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MLP_NIN = 5, MLP_NH = 64, MLP_NOUT = 2;
constexpr int OFF_W1 = 0, OFF_B1 = 320, OFF_W2 = 384, OFF_B2 = 4480, OFF_W3 = 4544,
              OFF_B3 = 8640, OFF_W4 = 8704, OFF_B4 = 8832, MLP_NPARAM = 8834;

// packed operand array, in units of one lane's bf16x8 (64 units per product)
constexpr int PK_P1 = 0;     // W1:   [mt 2][lane]
constexpr int PK_P2 = 128;   // W2:   [mt 2][kc 4][lane]
constexpr int PK_P3 = 640;   // W3:   [mt 2][kc 4][lane]
constexpr int PK_P4 = 1152;  // W4:   [kc 4][lane]          (rows >= 2 zero)
constexpr int PK_FWD = 1408; // end of the forward operands
constexpr int PK_T4 = 1408;  // W4^T: [mt 2][lane]          (k >= 2 zero)
constexpr int PK_T3 = 1536;  // W3^T: [mt 2][kc 4][lane]
constexpr int PK_T2 = 2048;  // W2^T: [mt 2][kc 4][lane]
constexpr int PK_ALL = 2560;

__host__ __device__ __forceinline__ int perm_in(int kc, int half, int s)
{
    const int r = 8 * (kc & 1) + s;
    return 32 * (kc >> 1) + 8 * (r >> 2) + 4 * half + (r & 3);
}

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float silu(float z)
{
    return z * frcp(1.0f + fexp2(-1.4426950408889634f * z));
}

// Saved forward state of 32 cells (training): the SiLU derivatives
// silu'(z) of the three hidden layers' pre-activations and the B operands
// fed to layers 2, 3, 4, both bf16 in the same register layout (layer l,
// tile mt, register r of the D layout at [4 l + 2 mt + r / 8][r % 8]).
struct MlpFwd {
    bf16x8 dz[12];
    bf16x8 h[12];
};

// silu(z) = z s and silu'(z) = s (1 + z (1 - s)), s = 1 / (1 + e^-z)
__device__ __forceinline__ float silu_keep(float z, float &dz)
{
    const float s = frcp(1.0f + fexp2(-1.4426950408889634f * z));
    dz = s * (1.0f + z * (1.0f - s));
    return z * s;
}

// Biases of the four layers (FP32), wherever they live (global or LDS).
struct MlpBias {
    const float *b1, *b2, *b3, *b4;
};

// Forward pass of 32 cells.  xb: this lane's B operand of layer 1 (features
// 0..4 of cell l%32 in lanes 0..31, zeros elsewhere).  pk: packed operands.
// Returns the two outputs of cell l%32 in lanes 0..31.
template <bool KEEP, typename PK>
__device__ __forceinline__ void mlp_forward32(const PK *pk, const MlpBias &bias, bf16x8 xb,
                                              MlpFwd &st, float &y0, float &y1)
{
    const int lane = threadIdx.x & 63, half = lane >> 5;
    const f32x16 zero = {};
    bf16x8 h[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const f32x16 acc = mfma32(pk[PK_P1 + mt * 64 + lane], xb, zero);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int n = 32 * mt + 8 * (r >> 2) + 4 * half + (r & 3);
            const float z = acc[r] + bias.b1[n];
            if (KEEP) {
                float dz;
                h[2 * mt + (r >> 3)][r & 7] = (__bf16)silu_keep(z, dz);
                st.dz[2 * mt + (r >> 3)][r & 7] = (__bf16)dz;
            } else {
                h[2 * mt + (r >> 3)][r & 7] = (__bf16)silu(z);
            }
        }
    }
    if (KEEP) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) st.h[kc] = h[kc];
    }
#pragma unroll
    for (int L = 0; L < 2; ++L) {
        const int P = L == 0 ? PK_P2 : PK_P3;
        const float *bl = L == 0 ? bias.b2 : bias.b3;
        bf16x8 hn[4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            f32x16 acc = zero;
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) acc = mfma32(pk[P + (mt * 4 + kc) * 64 + lane], h[kc], acc);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int n = 32 * mt + 8 * (r >> 2) + 4 * half + (r & 3);
                const float z = acc[r] + bl[n];
                if (KEEP) {
                    float dz;
                    hn[2 * mt + (r >> 3)][r & 7] = (__bf16)silu_keep(z, dz);
                    st.dz[4 * (L + 1) + 2 * mt + (r >> 3)][r & 7] = (__bf16)dz;
                } else {
                    hn[2 * mt + (r >> 3)][r & 7] = (__bf16)silu(z);
                }
            }
        }
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            h[kc] = hn[kc];
            if (KEEP) st.h[4 * (L + 1) + kc] = hn[kc];
        }
    }
    f32x16 acc = zero;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) acc = mfma32(pk[PK_P4 + kc * 64 + lane], h[kc], acc);
    y0 = acc[0] + bias.b4[0];
    y1 = acc[1] + bias.b4[1];
}

// Forward pass of the 64 cells of a wavefront (every lane takes part): sv
// holds this lane's five standardised features; returns this lane's two
// standardised outputs.  Two 32-cell passes, one after the other (the loop
// is kept rolled so that the two do not hold their operands at once): lanes
// 0..31 first, then the features of lanes 32..63 moved down and the outputs
// moved back up.
__device__ __forceinline__ void mlp_predict64(const bf16x8 *pk, const MlpBias &bias,
                                              const float sv[5], float &y0, float &y1)
{
    const int lane = threadIdx.x & 63;
    float up[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) up[k] = __shfl(sv[k], (lane + 32) & 63);
    float lo0 = 0.0f, lo1 = 0.0f, hi0 = 0.0f, hi1 = 0.0f;
#pragma nounroll
    for (int p = 0; p < 2; ++p) {
        bf16x8 x;
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = (__bf16)0.0f;
        if (lane < 32) {
#pragma unroll
            for (int k = 0; k < 5; ++k) x[k] = (__bf16)(p == 0 ? sv[k] : up[k]);
        }
        MlpFwd unused;
        float a0, a1;
        mlp_forward32<false>(pk, bias, x, unused, a0, a1);
        if (p == 0) {
            lo0 = a0;
            lo1 = a1;
        } else {
            hi0 = a0;
            hi1 = a1;
        }
    }
    const float sb0 = __shfl(hi0, lane & 31), sb1 = __shfl(hi1, lane & 31);
    y0 = lane < 32 ? lo0 : sb0;
    y1 = lane < 32 ? lo1 : sb1;
}

}  // namespace rtk
