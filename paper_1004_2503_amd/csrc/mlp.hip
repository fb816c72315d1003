// mlp.hip -- training and batch inference of the chemistry-surrogate network
// on gfx950 matrix cores, and the batch form of the exact per-cell chemistry
// operator that produces its training pairs.
//
// Training step = pack (FP32 master -> permuted bf16 operands) -> fused
// forward + backward per 32-sample chunk (one wavefront per block, every
// product on v_mfma_f32_32x32x16_bf16, the weight gradients accumulated in
// LDS in FP32) -> deterministic reduction of the per-block gradients -> Adam
// on the FP32 master.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "mlp_device.h"

namespace rtk {

// ------------------------------------------------------------ packing
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float *__restrict__ th,
                                                       __bf16 *__restrict__ pk)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= PK_ALL * 8) return;
    const int unit = e >> 3, s = e & 7;
    const int lane = unit & 63, half = lane >> 5, row = lane & 31;
    float v = 0.0f;
    if (unit < PK_P2) {                       // W1, A[out][in]
        const int mt = unit >> 6, in = 8 * half + s;
        if (in < MLP_NIN) v = th[OFF_W1 + (32 * mt + row) * MLP_NIN + in];
    } else if (unit < PK_P4) {                // W2, W3
        const bool l3 = unit >= PK_P3;
        const int g = (unit - (l3 ? PK_P3 : PK_P2)) >> 6, mt = g >> 2, kc = g & 3;
        const int off = l3 ? OFF_W3 : OFF_W2;
        v = th[off + (32 * mt + row) * MLP_NH + perm_in(kc, half, s)];
    } else if (unit < PK_T4) {                // W4 (2 rows)
        const int kc = (unit - PK_P4) >> 6;
        if (row < MLP_NOUT) v = th[OFF_W4 + row * MLP_NH + perm_in(kc, half, s)];
    } else if (unit < PK_T3) {                // W4^T: A[in][out]
        const int mt = (unit - PK_T4) >> 6, out = 8 * half + s;
        if (out < MLP_NOUT) v = th[OFF_W4 + out * MLP_NH + 32 * mt + row];
    } else {                                  // W3^T, W2^T: A[in][out = perm]
        const bool l2 = unit >= PK_T2;
        const int g = (unit - (l2 ? PK_T2 : PK_T3)) >> 6, mt = g >> 2, kc = g & 3;
        const int off = l2 ? OFF_W2 : OFF_W3;
        v = th[off + perm_in(kc, half, s) * MLP_NH + 32 * mt + row];
    }
    pk[e] = (__bf16)v;
}

// Batch sampling on the device: sample i of a step draws row
// floor(h / 2^32 * n) of the n training pairs, h the upper 32 bits of
// SplitMix64 (Steele, Lea & Flood 2014) at key + i; the step's key is
// SplitMix64 of seed XOR (step * 0xD1B54A32D192ED03).  n < 2^31.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t sample_row(uint64_t key, int64_t i, int64_t n)
{
    return int64_t(((splitmix64(key + uint64_t(i)) >> 32) * uint64_t(n)) >> 32);
}

struct SampleKey {
    int on;          // 0: sample i is row i
    uint64_t key;
    int64_t n;       // rows to draw from
};

__device__ __forceinline__ bf16x8 load_features(const float *__restrict__ X, int64_t smp,
                                                bool valid, int half)
{
    bf16x8 xb;
#pragma unroll
    for (int s = 0; s < 8; ++s) xb[s] = (__bf16)0.0f;
    if (valid && half == 0) {
#pragma unroll
        for (int f = 0; f < MLP_NIN; ++f) xb[f] = (__bf16)X[smp * MLP_NIN + f];
    }
    return xb;
}

// ------------------------------------------------------ batch inference
__global__ __launch_bounds__(256) void mlp_forward_kernel(const bf16x8 *__restrict__ pk,
                                                          const float *__restrict__ th,
                                                          const float *__restrict__ X,
                                                          int64_t B, float *__restrict__ Y)
{
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t nchunk = (B + 31) / 32;
    for (int64_t c = wave; c < nchunk; c += nw) {
        const int64_t smp = c * 32 + col;
        const bool valid = smp < B;
        MlpFwd st;
        float y0, y1;
        mlp_forward32<false>(pk, MlpBias{th + OFF_B1, th + OFF_B2, th + OFF_B3, th + OFF_B4},
                             load_features(X, smp, valid, half), st, y0, y1);
        if (valid && half == 0) {
            Y[smp * 2] = y0;
            Y[smp * 2 + 1] = y1;
        }
    }
}

// ------------------------------------------------ forward + backward
// Loss L = 1/(2B) sum (y - t)^2; each block writes the unscaled gradient of
// sum (y - t)^2 / 2 over its samples as one partial row, the reduction
// applies 1/B.  A block is GRAD_WAVES wavefronts that share the packed
// operands and the biases, staged in LDS once; wavefront w of block b takes
// the 32-sample chunks b GRAD_WAVES + w, + GRAD_WAVES gridDim.x, ...  The
// gradient of W3 (64 x 64) stays in the matrix cores' accumulator registers
// over all of a wavefront's chunks; that of W2 (64 x 64) and the small ones
// (W1, W4, the biases) go to an LDS area of the wavefront (W2 in registers
// too spilled to scratch: 512 registers per lane are not enough for both
// with the saved forward state).  Each wavefront transposes through LDS of
// its own, so no block barrier is needed inside the loop.  At the end the
// wavefronts' contributions are added in wavefront order (deterministic).
constexpr int GRAD_WAVES = 4, GRAD_THREADS = 64 * GRAD_WAVES;
// small gradients per wavefront: W1 (64 x 5), b1, b2, b3, W4 (2 x 64), b4
constexpr int GS_W1 = 0, GS_B1 = 320, GS_B2 = 384, GS_B3 = 448, GS_W4 = 512, GS_B4 = 640,
              GS_N = 642, GS_PAD = 644;
static_assert(GS_PAD >= GS_N && GS_PAD % 4 == 0, "small-gradient area");

struct GradWaveLds {
    __bf16 Gs[64][32];     // dL/dZ of a layer (neurons x samples), bf16
    __bf16 Hs[64][32];     // that layer's inputs (neurons x samples), bf16
    __bf16 G4s[2][32];     // output-layer dL/dY
    float g[GS_PAD];       // the small gradients
    float w2[MLP_NH * MLP_NH];   // the gradient of W2
};
static_assert(sizeof(GradWaveLds) % 16 == 0, "16-byte aligned per wavefront");

// orders the LDS accesses of one wavefront (its lanes exchange data through
// its own LDS area; the wavefront's LDS operations complete in order)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// index of parameter i among the small gradients (not W2, W3)
__device__ __forceinline__ int small_index(int i)
{
    if (i < OFF_B1) return GS_W1 + (i - OFF_W1);
    if (i < OFF_W2) return GS_B1 + (i - OFF_B1);
    if (i < OFF_W3) return GS_B2 + (i - OFF_B2);   // i >= OFF_B2 here
    if (i < OFF_W4) return GS_B3 + (i - OFF_B3);   // i >= OFF_B3 here
    if (i < OFF_B4) return GS_W4 + (i - OFF_W4);
    return GS_B4 + (i - OFF_B4);
}

__global__ __launch_bounds__(GRAD_THREADS) void mlp_grad_kernel(const bf16x8 *__restrict__ pk_g,
                                                                const float *__restrict__ th,
                                                                const float *__restrict__ X,
                                                                const float *__restrict__ Y,
                                                                int64_t B, SampleKey sk,
                                                                float *__restrict__ part,
                                                                double *__restrict__ lpart)
{
    __shared__ __attribute__((aligned(16))) bf16x8 s_pk[PK_ALL];
    __shared__ float s_bias[SURR_NBIAS];   // b1 | b2 | b3 | b4
    __shared__ __attribute__((aligned(16))) GradWaveLds s_w[GRAD_WAVES];
    __shared__ double s_loss[GRAD_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, col = lane & 31;
    for (int i = tid; i < PK_ALL; i += GRAD_THREADS) s_pk[i] = pk_g[i];
    for (int i = tid; i < 64; i += GRAD_THREADS) {
        s_bias[i] = th[OFF_B1 + i];
        s_bias[64 + i] = th[OFF_B2 + i];
        s_bias[128 + i] = th[OFF_B3 + i];
    }
    if (tid < 2) s_bias[192 + tid] = th[OFF_B4 + tid];
    GradWaveLds &W = s_w[wave];
    for (int i = lane; i < GS_PAD; i += 64) W.g[i] = 0.0f;
    for (int i = lane; i < MLP_NH * MLP_NH; i += 64) W.w2[i] = 0.0f;
    __syncthreads();
    const MlpBias mb{s_bias, s_bias + 64, s_bias + 128, s_bias + 192};

    const f32x16 zero = {};
    bf16x8 zero8, ones;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        zero8[s] = (__bf16)0.0f;
        ones[s] = (__bf16)(col == 0 ? 1.0f : 0.0f);
    }
    // dW3 as 2 x 2 tiles of 32 x 32 (mt: output neurons, nt: input
    // neurons) in the D layout
    f32x16 acc3[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc3[mt][nt] = zero;
    double lsum = 0.0;
    const int64_t nchunk = (B + 31) / 32;
    const int64_t nwv = int64_t(gridDim.x) * GRAD_WAVES;

    for (int64_t c = int64_t(blockIdx.x) * GRAD_WAVES + wave; c < nchunk; c += nwv) {
        const int64_t smp = c * 32 + col;
        const bool valid = smp < B;
        const int64_t row = sk.on ? sample_row(sk.key, smp, sk.n) : smp;
        const bf16x8 xb = load_features(X, row, valid, half);
        MlpFwd st;
        float y0, y1;
        mlp_forward32<true>(s_pk, mb, xb, st, y0, y1);
        float d0 = 0.0f, d1 = 0.0f;
        if (valid && half == 0) {
            d0 = y0 - Y[row * 2];
            d1 = y1 - Y[row * 2 + 1];
            lsum += double(d0) * d0 + double(d1) * d1;
        }

        // ---- output layer: G4 (2 x cells)
        bf16x8 g4 = zero8;
        if (half == 0) {
            g4[0] = (__bf16)d0;
            g4[1] = (__bf16)d1;
        }
        f32x16 G[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const f32x16 a = mfma32(s_pk[PK_T4 + mt * 64 + lane], g4, zero);
#pragma unroll
            for (int r = 0; r < 16; ++r)
                G[mt][r] = a[r] * float(st.dz[8 + 2 * mt + (r >> 3)][r & 7]);
        }
        wave_lds_sync();   // the previous chunk's reads of this area are done
        if (half == 0) {
            W.G4s[0][col] = (__bf16)d0;
            W.G4s[1][col] = (__bf16)d1;
        }
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
#pragma unroll
            for (int s = 0; s < 8; ++s) W.Hs[perm_in(kc, half, s)][col] = st.h[8 + kc][s];
        wave_lds_sync();
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x16 a = zero;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const bf16x8 A =
                    col < MLP_NOUT ? *(const bf16x8 *)&W.G4s[col][16 * kk + 8 * half] : zero8;
                const bf16x8 Bv = *(const bf16x8 *)&W.Hs[32 * nt + col][16 * kk + 8 * half];
                a = mfma32(A, Bv, a);
            }
            if (half == 0) {
                W.g[GS_W4 + 32 * nt + col] += a[0];
                W.g[GS_W4 + MLP_NH + 32 * nt + col] += a[1];
            }
        }
        {
            float s0 = d0, s1 = d1;
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) {
                s0 += __shfl_xor(s0, off);
                s1 += __shfl_xor(s1, off);
            }
            if (lane == 0) {
                W.g[GS_B4] += s0;
                W.g[GS_B4 + 1] += s1;
            }
        }

        // ---- hidden layers 3, 2, 1: G holds dL/dZ_L in the D layout
#pragma unroll
        for (int L = 3; L >= 1; --L) {
            const int gsB = L == 3 ? GS_B3 : (L == 2 ? GS_B2 : GS_B1);
            // G_L in bf16: the B operand of W_L^T G_L and, transposed
            // through LDS, the A operand of dW_L = G_L H_{L-1}^T and db_L
            bf16x8 gb[4];
#pragma unroll
            for (int kc = 0; kc < 4; ++kc)
#pragma unroll
                for (int s = 0; s < 8; ++s) gb[kc][s] = (__bf16)G[kc >> 1][8 * (kc & 1) + s];
            wave_lds_sync();
#pragma unroll
            for (int kc = 0; kc < 4; ++kc)
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int r = 8 * (kc & 1) + s;
                    W.Gs[32 * (kc >> 1) + 8 * (r >> 2) + 4 * half + (r & 3)][col] = gb[kc][s];
                }
            // gradient flowing to the previous layer: W_L^T G_L, times SiLU'
            f32x16 Gp[2];
            if (L > 1) {
                const int PT = L == 3 ? PK_T3 : PK_T2;
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
                    f32x16 a = zero;
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
                        a = mfma32(s_pk[PT + (mt * 4 + kc) * 64 + lane], gb[kc], a);
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        Gp[mt][r] = a[r] * float(st.dz[4 * (L - 2) + 2 * mt + (r >> 3)][r & 7]);
                }
            }
            if (L > 1) {
#pragma unroll
                for (int kc = 0; kc < 4; ++kc)
#pragma unroll
                    for (int s = 0; s < 8; ++s)
                        W.Hs[perm_in(kc, half, s)][col] = st.h[4 * (L - 2) + kc][s];
            } else {
                // inputs: rows 0..4 features, rows 5..31 zero
#pragma unroll
                for (int f = 0; f < 16; ++f)
                    W.Hs[16 * half + f][col] =
                        (__bf16)(half == 0 && f < 8 ? float(xb[f & 7]) : 0.0f);
            }
            wave_lds_sync();
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                bf16x8 A[2];
#pragma unroll
                for (int kk = 0; kk < 2; ++kk)
                    A[kk] = *(const bf16x8 *)&W.Gs[32 * mt + col][16 * kk + 8 * half];
                if (L == 3) {
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
                        for (int kk = 0; kk < 2; ++kk) {
                            const bf16x8 Bv =
                                *(const bf16x8 *)&W.Hs[32 * nt + col][16 * kk + 8 * half];
                            acc3[mt][nt] = mfma32(A[kk], Bv, acc3[mt][nt]);
                        }
                    }
                } else if (L == 2) {
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt) {
                        f32x16 a = zero;
#pragma unroll
                        for (int kk = 0; kk < 2; ++kk) {
                            const bf16x8 Bv =
                                *(const bf16x8 *)&W.Hs[32 * nt + col][16 * kk + 8 * half];
                            a = mfma32(A[kk], Bv, a);
                        }
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int rw = 32 * mt + 8 * (r >> 2) + 4 * half + (r & 3);
                            W.w2[rw * MLP_NH + 32 * nt + col] += a[r];
                        }
                    }
                } else {
                    f32x16 a = zero;
#pragma unroll
                    for (int kk = 0; kk < 2; ++kk) {
                        const bf16x8 Bv = *(const bf16x8 *)&W.Hs[col][16 * kk + 8 * half];
                        a = mfma32(A[kk], Bv, a);
                    }
                    if (col < MLP_NIN) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int rw = 32 * mt + 8 * (r >> 2) + 4 * half + (r & 3);
                            W.g[GS_W1 + rw * MLP_NIN + col] += a[r];
                        }
                    }
                }
                f32x16 a = zero;
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) a = mfma32(A[kk], ones, a);
                if (col == 0) {
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        W.g[gsB + 32 * mt + 8 * (r >> 2) + 4 * half + (r & 3)] += a[r];
                }
            }
            if (L > 1) {
                G[0] = Gp[0];
                G[1] = Gp[1];
            }
        }
    }

    // the block's partial row: dW3 added over the wavefronts in order in
    // the (now free) operand area, dW2 and the small gradients likewise
    __syncthreads();
    float *sW = reinterpret_cast<float *>(s_pk);   // dW3, 4096 floats
    static_assert(sizeof(bf16x8) * PK_ALL >= MLP_NH * MLP_NH * sizeof(float), "dW3 fits");
    for (int w = 0; w < GRAD_WAVES; ++w) {
        if (wave == w) {
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int rw = 32 * mt + 8 * (r >> 2) + 4 * half + (r & 3);
                        const int k = rw * MLP_NH + 32 * nt + col;
                        sW[k] = (w == 0 ? 0.0f : sW[k]) + acc3[mt][nt][r];
                    }
        }
        __syncthreads();
    }
    float *prow = part + size_t(blockIdx.x) * MLP_NPARAM;
    for (int i = tid; i < MLP_NPARAM; i += GRAD_THREADS) {
        float v;
        if (i >= OFF_W2 && i < OFF_B2) {
            const int k = i - OFF_W2;
            v = s_w[0].w2[k];
#pragma unroll
            for (int w = 1; w < GRAD_WAVES; ++w) v += s_w[w].w2[k];
        } else if (i >= OFF_W3 && i < OFF_B3) {
            v = sW[i - OFF_W3];
        } else {
            const int k = small_index(i);
            v = s_w[0].g[k];
#pragma unroll
            for (int w = 1; w < GRAD_WAVES; ++w) v += s_w[w].g[k];
        }
        prow[i] = v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) s_loss[wave] = lsum;
    __syncthreads();
    if (tid == 0) {
        double l = s_loss[0];
#pragma unroll
        for (int w = 1; w < GRAD_WAVES; ++w) l += s_loss[w];
        lpart[blockIdx.x] = l;
    }
}

// fixed-order reduction of the block gradients; grad = sum / B
// Sum of the per-block gradient partials, in a fixed order: a block of 16
// wavefronts owns 64 parameters (one per lane); wavefront w adds the partial
// rows w, w + 16, ... and the 16 wavefront sums are then combined in order.
// (One thread per parameter walking every row was latency-bound: 280 us
// for 1024 rows.)  Block 0 also reduces the loss partials.
constexpr int RED_WAVES = 16;
constexpr int RED_BLOCKS = (MLP_NPARAM + 63) / 64;
__global__ __launch_bounds__(64 * RED_WAVES) void mlp_reduce_kernel(
    const float *__restrict__ part, const double *__restrict__ lpart, int nblk, double invB,
    float *__restrict__ grad, double *__restrict__ loss, double *__restrict__ npart)
{
    __shared__ double s[RED_WAVES][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (j < MLP_NPARAM) {
#pragma unroll 4
        for (int b = w; b < nblk; b += RED_WAVES) acc += part[size_t(b) * MLP_NPARAM + j];
    }
    s[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        float g = 0.0f;
        if (j < MLP_NPARAM) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < RED_WAVES; ++k) t += s[k][lane];
            g = float(t * invB);
            grad[j] = g;
        }
        if (npart) {
            // this block's share of |grad|^2, summed by a fixed butterfly
            double q = double(g) * double(g);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
            if (lane == 0) npart[blockIdx.x] = q;
        }
    }
    if (blockIdx.x == 0 && loss) {
        __syncthreads();
        double l = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64 * RED_WAVES) l += lpart[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
        if (lane == 0) s[w][0] = l;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int k = 0; k < RED_WAVES; ++k) t += s[k][0];
            *loss = 0.5 * t * invB;
        }
    }
}

// Adam (Kingma & Ba 2015) on the FP32 master; c1, c2 are the bias corrections
// With npart, the gradient is first rescaled to global norm clip when its
// norm (from the nnp squared-norm partials of the reduction, added in a
// fixed order) exceeds clip.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ th,
                                                       float *__restrict__ m,
                                                       float *__restrict__ v,
                                                       const float *__restrict__ g, float lr,
                                                       float b1, float b2, float omb1,
                                                       float omb2, float eps, float c1, float c2,
                                                       const double *__restrict__ npart, int nnp,
                                                       double clip)
{
    __shared__ float s_scale;
    if (npart) {
        if (threadIdx.x < 64) {
            double q = 0.0;
            for (int k = threadIdx.x; k < nnp; k += 64) q += npart[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
            if (threadIdx.x == 0) s_scale = float(fmin(1.0, clip / (sqrt(q) + 1e-12)));
        }
        __syncthreads();
    }
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= MLP_NPARAM) return;
    const float gj = npart ? g[j] * s_scale : g[j];
    const float mj = b1 * m[j] + omb1 * gj;
    const float vj = b2 * v[j] + omb2 * gj * gj;
    m[j] = mj;
    v[j] = vj;
    th[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// ----------------------------------------- exact chemistry on a batch
// Constants of Phi for a batch of independent cells (rt_chem_apply,
// rt_mlp_pairs): the step's operator, FP64 below xhi_thr in the mixed form.
struct PhiK {
    int chem, mixed, adaptive, nsub;
    double csig, T_h, inv15kB, T_floor, sub_eps;
    float xhi_thr;
    ClumpLaw cl;
    ClumpLawD cld;
};

__device__ __forceinline__ int phi_cell(const PhiK &P, float nh, float d, float &N, float &x,
                                        float &T)
{
    if (P.mixed && x < P.xhi_thr) {
        const ChemK<double> K{double(d), double(d) / P.nsub, P.csig, P.T_h, P.T_floor,
                              P.sub_eps, P.inv15kB};
        double Nd = N, xd = x, Td = T, ad = 0.0, cR, cI;
        clump_f64(P.cld, double(nh), cR, cI);
        const int nc = chem_cell<double>(P.chem, P.nsub, P.adaptive, K, cR, cI, double(nh), Nd,
                                         xd, Td, ad);
        N = float(Nd);
        x = float(xd);
        T = float(Td);
        return nc;
    }
    const ChemK<float> K{d,          d / float(P.nsub), float(P.csig),   float(P.T_h),
                         float(P.T_floor), float(P.sub_eps), float(P.inv15kB)};
    float af = 0.0f, cR, cI;
    clump_f32(P.cl, nh, cR, cI);
    return chem_cell<float>(P.chem, P.nsub, P.adaptive, K, cR, cI, nh, N, x, T, af);
}

__global__ __launch_bounds__(256) void chem_batch_kernel(int64_t n, const float *__restrict__ nH,
                                                         float *__restrict__ N,
                                                         float *__restrict__ xHI,
                                                         float *__restrict__ T,
                                                         const float *__restrict__ dt, PhiK P,
                                                         int32_t *__restrict__ ncyc)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    float Nf = N[i], xf = xHI[i], Tf = T[i];
    const int nc = phi_cell(P, nH[i], dt[i], Nf, xf, Tf);
    N[i] = Nf;
    xHI[i] = xf;
    T[i] = Tf;
    if (ncyc) ncyc[i] = nc;
}

// ------------------------------------------------- training pairs
// Features of a cell: log10 of nH, max(xHI, FLOOR), T, max(N, FLOOR), dt;
// with the exact operator applied to a copy: the targets u = asinh(d /
// DSCALE) of the changes d = log10(xHI'/xHI), log10(T'/T) (xHI floored
// likewise) and the end values log10 xHI', log10 T'.  FP64 logarithms.
constexpr double MLP_FLOOR = 1e-30;
constexpr double MLP_DSCALE = 1e-3;

__global__ __launch_bounds__(256) void mlp_pairs_kernel(int64_t n, const float *__restrict__ nH,
                                                        const float *__restrict__ N,
                                                        const float *__restrict__ xHI,
                                                        const float *__restrict__ T,
                                                        const float *__restrict__ dt, PhiK P,
                                                        float *__restrict__ X,
                                                        float *__restrict__ U,
                                                        float *__restrict__ Yend,
                                                        int32_t *__restrict__ ncyc)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const float nh = nH[i], n0 = N[i], x0 = xHI[i], t0 = T[i], d = dt[i];
    const double lx0 = log10(fmax(double(x0), MLP_FLOOR)), lt0 = log10(double(t0));
    if (X) {
        X[i * 5 + 0] = float(log10(double(nh)));
        X[i * 5 + 1] = float(lx0);
        X[i * 5 + 2] = float(lt0);
        X[i * 5 + 3] = float(log10(fmax(double(n0), MLP_FLOOR)));
        X[i * 5 + 4] = float(log10(double(d)));
    }
    if (!U && !Yend && !ncyc) return;
    float n1 = n0, x1 = x0, t1 = t0;
    const int nc = phi_cell(P, nh, d, n1, x1, t1);
    const double lx1 = log10(fmax(double(x1), MLP_FLOOR)), lt1 = log10(double(t1));
    if (U) {
        U[i * 2 + 0] = float(asinh((lx1 - lx0) / MLP_DSCALE));
        U[i * 2 + 1] = float(asinh((lt1 - lt0) / MLP_DSCALE));
    }
    if (Yend) {
        Yend[i * 2 + 0] = float(lx1);
        Yend[i * 2 + 1] = float(lt1);
    }
    if (ncyc) ncyc[i] = nc;
}

// ------------------------------------------------- standardisation
// Column moments of an (n, d) FP32 array, d <= MOM_MAXD, in FP64 and in a
// fixed order: block b sums rows [b n / MOM_BLOCKS, (b+1) n / MOM_BLOCKS)
// thread by thread (stride 256) and then over its threads by a fixed
// tree; one block adds the block partials in order.  Pass 0: sums, minima,
// maxima; pass 1: sums of squared deviations from the mean.
constexpr int MOM_BLOCKS = 128, MOM_MAXD = 8;

__global__ __launch_bounds__(256) void mlp_moments_kernel(const float *__restrict__ A, int64_t n,
                                                          int d, const double *__restrict__ stats,
                                                          double *__restrict__ part)
{
    __shared__ double s_a[MOM_MAXD][256];
    __shared__ float s_lo[MOM_MAXD][256], s_hi[MOM_MAXD][256];
    const int t = threadIdx.x;
    const int64_t r0 = int64_t(blockIdx.x) * n / MOM_BLOCKS;
    const int64_t r1 = int64_t(blockIdx.x + 1) * n / MOM_BLOCKS;
    double mu[MOM_MAXD], acc[MOM_MAXD];
    float lo[MOM_MAXD], hi[MOM_MAXD];
#pragma unroll
    for (int k = 0; k < MOM_MAXD; ++k) {
        mu[k] = (stats && k < d) ? stats[k] : 0.0;
        acc[k] = 0.0;
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    // one pass over the rows, every column of a row at once
    for (int64_t r = r0 + t; r < r1; r += 256) {
#pragma unroll
        for (int k = 0; k < MOM_MAXD; ++k) {
            if (k >= d) break;
            const float v = A[r * d + k];
            if (stats) {
                const double e = double(v) - mu[k];
                acc[k] += e * e;
            } else {
                acc[k] += double(v);
                lo[k] = fminf(lo[k], v);
                hi[k] = fmaxf(hi[k], v);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < MOM_MAXD; ++k) {
        s_a[k][t] = acc[k];
        s_lo[k][t] = lo[k];
        s_hi[k][t] = hi[k];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int k = 0; k < MOM_MAXD; ++k) {
                s_a[k][t] += s_a[k][t + h];
                s_lo[k][t] = fminf(s_lo[k][t], s_lo[k][t + h]);
                s_hi[k][t] = fmaxf(s_hi[k][t], s_hi[k][t + h]);
            }
        }
        __syncthreads();
    }
    if (t < d) {
        double *row = part + size_t(blockIdx.x) * 3 * MOM_MAXD;
        row[t] = s_a[t][0];
        row[MOM_MAXD + t] = double(s_lo[t][0]);
        row[2 * MOM_MAXD + t] = double(s_hi[t][0]);
    }
}

// stats: mean[d], sd[d], min[d], max[d]; pass 0 fills mean, min, max, pass 1
// sd = sqrt(sum of squares / (n - 1)), at least 1e-6 (1 for n = 1).
__global__ __launch_bounds__(64) void mlp_moments_final_kernel(const double *__restrict__ part,
                                                               int64_t n, int d, int pass,
                                                               double *__restrict__ stats)
{
    const int k = threadIdx.x;
    if (k >= d) return;
    double acc = 0.0, lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < MOM_BLOCKS; ++b) {
        const double *row = part + size_t(b) * 3 * MOM_MAXD;
        acc += row[k];
        lo = fmin(lo, row[MOM_MAXD + k]);
        hi = fmax(hi, row[2 * MOM_MAXD + k]);
    }
    if (pass == 0) {
        stats[k] = acc / double(n);
        stats[2 * d + k] = lo;
        stats[3 * d + k] = hi;
    } else {
        stats[d + k] = n > 1 ? fmax(sqrt(acc / double(n - 1)), 1e-6) : 1.0;
    }
}

__global__ __launch_bounds__(256) void mlp_standardize_kernel(const float *__restrict__ A,
                                                              int64_t n, int d,
                                                              const double *__restrict__ stats,
                                                              float *__restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n * d) return;
    const int k = int(i % d);
    out[i] = float((double(A[i]) - stats[k]) / stats[d + k]);
}

// ------------------------------------------------- prediction
// Raw features -> standardised (norm: mu_in[5] sd_in[5] mu_out[2] sd_out[2],
// FP32) -> network -> u = y sd_out + mu_out -> end values log10 xHI' =
// f1 + DSCALE sinh u0, log10 T' = f2 + DSCALE sinh u1 (Y, optional); with
// targets U (encoded changes, optional), the block's sum of squared
// standardised errors (y - (U - mu_out) / sd_out)^2 over both outputs.
struct PredNorm {
    float v[14];
};

__global__ __launch_bounds__(256) void mlp_predict_kernel(const bf16x8 *__restrict__ pk,
                                                          const float *__restrict__ th,
                                                          PredNorm nm,
                                                          const float *__restrict__ X,
                                                          int64_t B, float *__restrict__ Y,
                                                          const float *__restrict__ U,
                                                          double *__restrict__ lpart)
{
    __shared__ double s_l[4];
    const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    const int wave = threadIdx.x >> 6;
    const int64_t wv = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t nchunk = (B + 31) / 32;
    double lsum = 0.0;
    for (int64_t c = wv; c < nchunk; c += nw) {
        const int64_t smp = c * 32 + col;
        const bool valid = smp < B;
        bf16x8 xb;
        float f1 = 0.0f, f2 = 0.0f;
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2) xb[s2] = (__bf16)0.0f;
        if (valid && half == 0) {
#pragma unroll
            for (int f = 0; f < MLP_NIN; ++f)
                xb[f] = (__bf16)((X[smp * MLP_NIN + f] - nm.v[f]) / nm.v[5 + f]);
            f1 = X[smp * MLP_NIN + 1];
            f2 = X[smp * MLP_NIN + 2];
        }
        MlpFwd st;
        float y0, y1;
        mlp_forward32<false>(pk, MlpBias{th + OFF_B1, th + OFF_B2, th + OFF_B3, th + OFF_B4}, xb,
                             st, y0, y1);
        if (valid && half == 0) {
            if (Y) {
                const double u0 = double(y0) * nm.v[12] + nm.v[10];
                const double u1 = double(y1) * nm.v[13] + nm.v[11];
                Y[smp * 2] = float(double(f1) + MLP_DSCALE * sinh(u0));
                Y[smp * 2 + 1] = float(double(f2) + MLP_DSCALE * sinh(u1));
            }
            if (U) {
                const double e0 = double(y0) - (double(U[smp * 2]) - nm.v[10]) / nm.v[12];
                const double e1 = double(y1) - (double(U[smp * 2 + 1]) - nm.v[11]) / nm.v[13];
                lsum += e0 * e0 + e1 * e1;
            }
        }
    }
    if (lpart) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
        if (lane == 0) s_l[wave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) lpart[blockIdx.x] = ((s_l[0] + s_l[1]) + s_l[2]) + s_l[3];
    }
}

// out = scale * sum of the n partials, in a fixed order: lane l adds the
// partials l, l + 64, ..., then a fixed butterfly combines the lanes
__global__ __launch_bounds__(64) void mlp_sum_kernel(const double *__restrict__ part, int n,
                                                     double scale, double *__restrict__ out)
{
    double t = 0.0;
    for (int b = threadIdx.x; b < n; b += 64) t += part[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (threadIdx.x == 0) *out = t * scale;
}

hipError_t launch_mlp_pack(const float *theta, __bf16 *pk, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((PK_ALL * 8 + 255) / 256), dim3(256), 0, s, theta,
                       pk);
    return hipGetLastError();
}

}  // namespace rtk

using namespace rtk;

struct rt_mlp {
    hipStream_t stream = nullptr;
    int nblk = 0;
    __bf16 *pk = nullptr;
    float *part = nullptr;     // gradient partials; also the moment and loss partials
    double *lpart = nullptr;
    double *npart = nullptr;   // squared-norm partials of the reduction
    float *grad = nullptr;     // rt_mlp_train's gradient
};

namespace {
constexpr double KB_ = 1.380649e-16;
constexpr double EV_ = 1.602176634e-12;

int pack(rt_mlp *m, const float *theta)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((PK_ALL * 8 + 255) / 256), dim3(256), 0, m->stream,
                       theta, m->pk);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}
}  // namespace

extern "C" int rt_mlp_create(int32_t grad_blocks, void *hip_stream, rt_mlp **out)
{
    if (!out) return RT_E_ARG;
    *out = nullptr;
    if (grad_blocks < 1 || grad_blocks > 65536) return RT_E_ARG;
    rt_mlp *m = new (std::nothrow) rt_mlp();
    if (!m) return RT_E_NOMEM;
    m->stream = static_cast<hipStream_t>(hip_stream);
    m->nblk = grad_blocks;
    if (hipMalloc(&m->pk, size_t(PK_ALL) * 8 * sizeof(__bf16)) != hipSuccess ||
        hipMalloc(&m->part, size_t(grad_blocks) * MLP_NPARAM * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->lpart, size_t(grad_blocks) * sizeof(double)) != hipSuccess ||
        hipMalloc(&m->npart, size_t(RED_BLOCKS) * sizeof(double)) != hipSuccess ||
        hipMalloc(&m->grad, size_t(MLP_NPARAM) * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        if (m->pk) (void)hipFree(m->pk);
        if (m->part) (void)hipFree(m->part);
        if (m->lpart) (void)hipFree(m->lpart);
        if (m->npart) (void)hipFree(m->npart);
        delete m;
        return RT_E_NOMEM;
    }
    *out = m;
    return RT_OK;
}

extern "C" int rt_mlp_destroy(rt_mlp *m)
{
    if (!m) return RT_E_STATE;
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(m->pk);
    (void)hipFree(m->part);
    (void)hipFree(m->lpart);
    (void)hipFree(m->npart);
    (void)hipFree(m->grad);
    delete m;
    return RT_OK;
}

extern "C" int rt_mlp_forward(rt_mlp *m, const float *theta, const float *X, int64_t B,
                              float *Y)
{
    if (!m) return RT_E_STATE;
    if (B < 0 || (B > 0 && (!theta || !X || !Y))) return RT_E_ARG;
    if (B == 0) return RT_OK;
    if (pack(m, theta) != RT_OK) return RT_E_HIP;
    const int64_t nchunk = (B + 31) / 32;
    const int64_t blocks = (nchunk + 3) / 4 < 16384 ? (nchunk + 3) / 4 : 16384;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(unsigned(blocks)), dim3(256), 0, m->stream,
                       reinterpret_cast<const bf16x8 *>(m->pk), theta, X, B, Y);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

extern "C" int rt_mlp_grad(rt_mlp *m, const float *theta, const float *X, const float *Y,
                           int64_t B, float *grad, double *loss_dev)
{
    if (!m) return RT_E_STATE;
    if (B < 1 || !theta || !X || !Y || !grad) return RT_E_ARG;
    if (pack(m, theta) != RT_OK) return RT_E_HIP;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(m->nblk), dim3(GRAD_THREADS), 0, m->stream,
                       reinterpret_cast<const bf16x8 *>(m->pk), theta, X, Y, B,
                       SampleKey{0, 0ull, 0}, m->part, m->lpart);
    if (hipGetLastError() != hipSuccess) return RT_E_HIP;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(RED_BLOCKS), dim3(64 * RED_WAVES), 0, m->stream,
                       m->part, m->lpart, m->nblk, 1.0 / double(B), grad, loss_dev,
                       static_cast<double *>(nullptr));
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

// ---------------------------------------------- allocation-free gradient
// The packed operands, the loss partials and the per-block gradient partials
// of rt_mlp_grad_noalloc live in one fixed array per device, reserved when
// the library's code object is loaded.  Host code never passes the array's
// name to a kernel (in host code it is only a stand-in for the symbol): its
// device address is looked up once per device and used from then on.
namespace {
constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t NA_PK_BYTES = round256(size_t(PK_ALL) * 8 * sizeof(__bf16));
constexpr size_t NA_LOSS_BYTES = round256(size_t(RT_MLP_NOALLOC_BLOCKS) * sizeof(double));
constexpr size_t NA_PART_BYTES = size_t(RT_MLP_NOALLOC_BLOCKS) * MLP_NPARAM * sizeof(float);
constexpr size_t NA_BYTES = NA_PK_BYTES + NA_LOSS_BYTES + NA_PART_BYTES;
static_assert(NA_BYTES == size_t(RT_MLP_NOALLOC_BYTES), "rt.h states the scratch size");
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {
constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
unsigned char *na_ptr[NA_MAX_DEVICES] = {};

// Device address of `scratch` on the device of `stream` (the current device
// for the null stream), looked up with that device current on the first
// call for it.
int noalloc_scratch(hipStream_t stream, unsigned char **out)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return RT_E_HIP;
    int dev = cur;
    if (stream && hipStreamGetDevice(stream, &dev) != hipSuccess) return RT_E_HIP;
    if (dev < 0 || dev >= NA_MAX_DEVICES) return RT_E_HIP;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        if (dev != cur && hipSetDevice(dev) != hipSuccess) return RT_E_HIP;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur && hipSetDevice(cur) != hipSuccess) return RT_E_HIP;
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return RT_E_HIP;
        }
        na_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = na_ptr[dev];
    return RT_OK;
}
}  // namespace

extern "C" int rt_mlp_grad_noalloc(int32_t grad_blocks, const float *theta, const float *X,
                                   const float *Y, int64_t B, float *grad, double *loss_dev,
                                   void *hip_stream)
{
    if (grad_blocks < 1) return RT_E_ARG;
    if (grad_blocks > RT_MLP_NOALLOC_BLOCKS) return RT_E_SCRATCH;
    if (B < 1 || !theta || !X || !Y || !grad) return RT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    unsigned char *base = nullptr;
    const int rc = noalloc_scratch(s, &base);
    if (rc != RT_OK) return rc;
    __bf16 *pk = reinterpret_cast<__bf16 *>(base);
    double *lpart = reinterpret_cast<double *>(base + NA_PK_BYTES);
    float *part = reinterpret_cast<float *>(base + NA_PK_BYTES + NA_LOSS_BYTES);
    // every partial row and loss partial is written by its block before the
    // reduction reads it, and pk by the packing kernel: nothing to clear
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((PK_ALL * 8 + 255) / 256), dim3(256), 0, s, theta,
                       pk);
    if (hipGetLastError() != hipSuccess) return RT_E_HIP;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(grad_blocks), dim3(GRAD_THREADS), 0, s,
                       reinterpret_cast<const bf16x8 *>(pk), theta, X, Y, B,
                       SampleKey{0, 0ull, 0}, part, lpart);
    if (hipGetLastError() != hipSuccess) return RT_E_HIP;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(RED_BLOCKS), dim3(64 * RED_WAVES), 0, s, part,
                       lpart, grad_blocks, 1.0 / double(B), grad, loss_dev,
                       static_cast<double *>(nullptr));
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

extern "C" int rt_mlp_adam(rt_mlp *m, float *theta, float *mom1, float *mom2,
                           const float *grad, int64_t step, double lr, double beta1,
                           double beta2, double eps)
{
    if (!m) return RT_E_STATE;
    if (!theta || !mom1 || !mom2 || !grad || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0) ||
        !(beta1 < 1.0) || !(beta2 >= 0.0) || !(beta2 < 1.0) || !(eps >= 0.0))
        return RT_E_ARG;
    const double c1 = 1.0 - pow(beta1, double(step));
    const double c2 = 1.0 - pow(beta2, double(step));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0,
                       m->stream, theta, mom1, mom2, grad, float(lr), float(beta1),
                       float(beta2), float(1.0 - beta1), float(1.0 - beta2), float(eps),
                       float(c1), float(c2), static_cast<const double *>(nullptr), 0, 0.0);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

namespace {
// the chemistry fields rt_chem_apply and rt_mlp_pairs read
int check_chem(const rt_params *p, int32_t nsub)
{
    if (!p) return RT_E_ARG;
    if (nsub < 1 || nsub > 4096) return RT_E_ARG;
    if (p->chem < RT_CHEM_FULL || p->chem > RT_CHEM_FROZEN) return RT_E_ARG;
    if (p->prec != RT_PREC_FP32 && p->prec != RT_PREC_MIXED) return RT_E_ARG;
    if (p->sub != RT_SUB_FIXED && p->sub != RT_SUB_ADAPTIVE) return RT_E_ARG;
    if (p->sub == RT_SUB_ADAPTIVE && !(p->sub_eps > 0.0 && p->sub_eps <= 1.0)) return RT_E_ARG;
    if (!(p->c_cms > 0.0) || !(p->sigma_n > 0.0) || !(p->sigma_e > 0.0) ||
        !(p->egamma_eV > 0.0) || !(p->T_floor >= 0.0))
        return RT_E_ARG;
    if (check_clump(*p) != RT_OK) return RT_E_ARG;
    return RT_OK;
}

PhiK make_phik(const rt_params &p, int32_t nsub)
{
    const double eheat = (p.sigma_e * p.egamma_eV / p.sigma_n - 13.6) * EV_;
    PhiK k;
    k.chem = p.chem;
    k.mixed = p.prec == RT_PREC_MIXED ? 1 : 0;
    k.adaptive = p.sub == RT_SUB_ADAPTIVE ? 1 : 0;
    k.nsub = nsub;
    k.csig = p.c_cms * p.sigma_n;
    k.T_h = eheat / (1.5 * KB_);
    k.inv15kB = 1.0 / (1.5 * KB_);
    k.T_floor = p.T_floor;
    k.sub_eps = p.sub_eps;
    k.xhi_thr = float(p.xhi_fp64_thr);
    k.cl = make_clump_law(p);
    k.cld = make_clump_law_d(p);
    return k;
}
}  // namespace

extern "C" int rt_chem_apply(const rt_params *p, int64_t n, const float *nH, float *N,
                             float *xHI, float *T, const float *dt, int32_t nsub,
                             int32_t *ncycles, void *hip_stream)
{
    if (check_chem(p, nsub) != RT_OK || n < 0) return RT_E_ARG;
    if (n == 0) return RT_OK;
    if (!nH || !N || !xHI || !T || !dt) return RT_E_ARG;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return RT_E_ARG;
    hipLaunchKernelGGL(chem_batch_kernel, dim3(unsigned(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), n, nH, N, xHI, T, dt,
                       make_phik(*p, nsub), ncycles);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

extern "C" int rt_mlp_pairs(const rt_params *p, int64_t n, const float *nH, const float *N,
                            const float *xHI, const float *T, const float *dt, int32_t nsub,
                            float *X, float *U, float *Yend, int32_t *ncycles, void *hip_stream)
{
    if (check_chem(p, nsub) != RT_OK || n < 0) return RT_E_ARG;
    if (n == 0) return RT_OK;
    if (!nH || !N || !xHI || !T || !dt || (!X && !U && !Yend && !ncycles)) return RT_E_ARG;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff || n > (int64_t(1) << 40)) return RT_E_ARG;
    hipLaunchKernelGGL(mlp_pairs_kernel, dim3(unsigned(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), n, nH, N, xHI, T, dt,
                       make_phik(*p, nsub), X, U, Yend, ncycles);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

extern "C" int rt_mlp_standardize(rt_mlp *m, const float *A, int64_t n, int32_t d, float *out,
                                  double *stats)
{
    if (!m) return RT_E_STATE;
    if (n < 1 || d < 1 || d > MOM_MAXD || !A || !out || !stats) return RT_E_ARG;
    if (n > (int64_t(1) << 40)) return RT_E_ARG;
    // the moment partials (MOM_BLOCKS rows of 3 MOM_MAXD doubles) fit in the
    // gradient partials of one block
    static_assert(size_t(MOM_BLOCKS) * 3 * MOM_MAXD * sizeof(double) <=
                      size_t(MLP_NPARAM) * sizeof(float),
                  "moment partials fit in one gradient partial row");
    double *part = reinterpret_cast<double *>(m->part);
    hipStream_t s = m->stream;
    hipLaunchKernelGGL(mlp_moments_kernel, dim3(MOM_BLOCKS), dim3(256), 0, s, A, n, int(d),
                       static_cast<const double *>(nullptr), part);
    hipLaunchKernelGGL(mlp_moments_final_kernel, dim3(1), dim3(64), 0, s,
                       static_cast<const double *>(part), n, int(d), 0, stats);
    hipLaunchKernelGGL(mlp_moments_kernel, dim3(MOM_BLOCKS), dim3(256), 0, s, A, n, int(d),
                       static_cast<const double *>(stats), part);
    hipLaunchKernelGGL(mlp_moments_final_kernel, dim3(1), dim3(64), 0, s,
                       static_cast<const double *>(part), n, int(d), 1, stats);
    const int64_t blocks = (n * d + 255) / 256;
    if (blocks > 0x7fffffff) return RT_E_ARG;
    hipLaunchKernelGGL(mlp_standardize_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, A, n,
                       int(d), static_cast<const double *>(stats), out);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}

namespace {
// learning rate of step s (1-based): a linear rise over the first
// max(1, floor(warmup total)) steps, then a cosine decay to lr_floor
double lr_at(const rt_mlp_train_opts &o, int64_t s)
{
    const int64_t nw = std::max<int64_t>(int64_t(o.warmup * double(o.total_steps)), 1);
    if (s <= nw) return o.lr * double(s) / double(nw);
    const double ph = double(s - nw) / double(std::max<int64_t>(o.total_steps - nw, 1));
    return o.lr * 0.5 * (1.0 + cos(M_PI * ph)) + o.lr_floor;
}
}  // namespace

extern "C" int rt_mlp_train(rt_mlp *m, float *theta, float *mom1, float *mom2, const float *X,
                            const float *Y, int64_t n, const rt_mlp_train_opts *o,
                            int64_t step0, int64_t nsteps, double *loss_dev)
{
    if (!m) return RT_E_STATE;
    if (!theta || !mom1 || !mom2 || !X || !Y || !o) return RT_E_ARG;
    if (n < 1 || n >= (int64_t(1) << 31)) return RT_E_ARG;
    if (o->batch < 1 || o->total_steps < 1 || !(o->lr > 0.0) || !(o->warmup >= 0.0) ||
        !(o->warmup < 1.0) || !(o->lr_floor >= 0.0) || !isfinite(o->clip) ||
        !(o->beta1 >= 0.0) || !(o->beta1 < 1.0) || !(o->beta2 >= 0.0) || !(o->beta2 < 1.0) ||
        !(o->eps >= 0.0))
        return RT_E_ARG;
    if (step0 < 0 || nsteps < 0 || step0 + nsteps > o->total_steps) return RT_E_ARG;
    hipStream_t s = m->stream;
    const bool clip = o->clip > 0.0;
    for (int64_t st = step0 + 1; st <= step0 + nsteps; ++st) {
        const SampleKey sk{1, splitmix64(o->seed ^ (uint64_t(st) * 0xD1B54A32D192ED03ull)), n};
        if (pack(m, theta) != RT_OK) return RT_E_HIP;
        hipLaunchKernelGGL(mlp_grad_kernel, dim3(m->nblk), dim3(GRAD_THREADS), 0, s,
                           reinterpret_cast<const bf16x8 *>(m->pk), static_cast<const float *>(theta),
                           X, Y, o->batch, sk, m->part, m->lpart);
        hipLaunchKernelGGL(mlp_reduce_kernel, dim3(RED_BLOCKS), dim3(64 * RED_WAVES), 0, s,
                           static_cast<const float *>(m->part),
                           static_cast<const double *>(m->lpart), m->nblk,
                           1.0 / double(o->batch), m->grad, loss_dev,
                           clip ? m->npart : static_cast<double *>(nullptr));
        const double c1 = 1.0 - pow(o->beta1, double(st));
        const double c2 = 1.0 - pow(o->beta2, double(st));
        hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s,
                           theta, mom1, mom2, static_cast<const float *>(m->grad),
                           float(lr_at(*o, st)), float(o->beta1), float(o->beta2),
                           float(1.0 - o->beta1), float(1.0 - o->beta2), float(o->eps),
                           float(c1), float(c2),
                           clip ? static_cast<const double *>(m->npart) : nullptr, RED_BLOCKS,
                           o->clip);
        if (hipGetLastError() != hipSuccess) return RT_E_HIP;
    }
    return RT_OK;
}

extern "C" int rt_mlp_predict(rt_mlp *m, const float *theta, const float *norm, const float *X,
                              int64_t n, float *Y, const float *U, double *loss_dev)
{
    if (!m) return RT_E_STATE;
    if (n < 0 || !theta || !norm || (n > 0 && !X) || (!Y && !loss_dev) ||
        (loss_dev && !U))
        return RT_E_ARG;
    PredNorm nm;
    for (int k = 0; k < 14; ++k) {
        nm.v[k] = norm[k];
        if (!isfinite(nm.v[k])) return RT_E_ARG;
    }
    for (int k = 5; k < 10; ++k)
        if (!(nm.v[k] > 0.0f)) return RT_E_ARG;
    if (!(nm.v[12] > 0.0f) || !(nm.v[13] > 0.0f)) return RT_E_ARG;
    if (n == 0) {
        if (!loss_dev) return RT_OK;
        hipLaunchKernelGGL(mlp_sum_kernel, dim3(1), dim3(64), 0, m->stream,
                           static_cast<const double *>(m->lpart), 0, 0.0, loss_dev);
        return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
    }
    if (pack(m, theta) != RT_OK) return RT_E_HIP;
    const int64_t nchunk = (n + 31) / 32;
    // the loss partials (one double per block) live in the gradient partials
    const int64_t cap = loss_dev ? int64_t(MLP_NPARAM) / 2 : 16384;
    const int64_t want = (nchunk + 3) / 4;
    const int64_t blocks = want < cap ? want : cap;
    double *lp = loss_dev ? reinterpret_cast<double *>(m->part) : nullptr;
    hipLaunchKernelGGL(mlp_predict_kernel, dim3(unsigned(blocks)), dim3(256), 0, m->stream,
                       reinterpret_cast<const bf16x8 *>(m->pk), theta, nm, X, n, Y,
                       loss_dev ? U : nullptr, lp);
    if (loss_dev)
        hipLaunchKernelGGL(mlp_sum_kernel, dim3(1), dim3(64), 0, m->stream,
                           static_cast<const double *>(lp), int(blocks),
                           1.0 / (2.0 * double(n)), loss_dev);
    return hipGetLastError() == hipSuccess ? RT_OK : RT_E_HIP;
}
