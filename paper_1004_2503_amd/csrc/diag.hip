// Run diagnostics on gfx950: the distribution of cells over density and
// neutral fraction or photoionisation rate (Sec. 3.1.5), with the per-density
// bin sums that give the mean curves.
//
// Also the equilibrium neutral fraction under the self-shielding intensity
// models of the same section (one thread per element, FP64).
//
// One streaming pass over nH and the chosen quantity (8 bytes per cell).
// Each block keeps a private histogram in LDS (integer atomics) and exact
// fixed-point per-density-bin sums (see hist_kernel); blocks then add their
// non-zero bins to the global result.  Bin decisions are exact:
// an FP32 logarithm proposes the bin and comparisons against the FP64 edges
// settle it.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rt_device.h"
#include "rt_internal.h"

namespace rtk {

// edges[0..nbx] then edges[nbx+1 .. nbx+nby+1] in dynamic LDS
__device__ __forceinline__ int find_bin(double v, float lv, const double *e, int nb, float lo,
                                        float inv_w)
{
    float t = (lv - lo) * inv_w;
    t = fminf(fmaxf(t, 0.0f), float(nb - 1));   // also maps -inf (v = 0) to 0
    int k = int(t);
    while (k > 0 && v < e[k]) --k;
    while (k < nb - 1 && v >= e[k + 1]) ++k;
    return k;
}

// Sums of q per density bin are exact, hence independent of the order of
// the additions: every value is a float (xHI, or N for the rate, whose bin
// sum is multiplied by c sigma_n at the end), i.e. m 2^(s - 149) with an
// integer m < 2^24 and 0 <= s <= 253, and it is added as the integer
// m 2^s, split over two 32-bit-aligned limbs of a fixed-point accumulator
// (HLIMBS limbs of 64 bits per bin, 32 bits of headroom each: fewer than
// 2^32 cells cannot overflow one).  Blocks add their LDS limbs to the
// global ones with integer atomics; hist_sum_kernel propagates the carries
// and converts.  Negative or non-finite values are counted in a slot of
// their own and turn the bin's sum into NaN.  Counts are integers, added
// with atomics (exact in any order).
constexpr int HIST_THREADS = 256;
constexpr int HLIMBS = 9;            // limb k holds bits 32k .. 32k + 31 of m 2^s
constexpr int HSLOT = HLIMBS + 1;    // + the count of values without an exact sum

// v as an integer on the fixed-point grid: v = p 2^(32 k - 149) with
// p < 2^56; p = 0 for +-0.  Returns false for a negative or non-finite v.
__device__ __forceinline__ bool fixed_point(float v, int &k, unsigned long long &p)
{
    const uint32_t u = __float_as_uint(v);
    k = 0;
    p = 0ull;
    if (u == 0u || u == 0x80000000u) return true;      // +0, -0
    if (u >= 0x7f800000u) return false;                 // inf, NaN, negative
    const uint32_t e = u >> 23, mant = u & 0x7fffffu;
    const uint32_t m = e ? (mant | 0x800000u) : mant;
    const uint32_t s = e ? e - 1u : 0u;                 // v = m 2^(s - 149)
    k = int(s >> 5);
    p = (unsigned long long)m << (s & 31u);
    return true;
}

// Adds p 2^(32 k - 149) (p < 2^59: up to eight values of one limb) to a
// bin's limbs.
__device__ __forceinline__ void limb_add(unsigned long long *acc, int k, unsigned long long p)
{
    if (p & 0xffffffffull) atomicAdd(&acc[k], p & 0xffffffffull);
    if (p >> 32) atomicAdd(&acc[k + 1], p >> 32);
}

__global__ __launch_bounds__(HIST_THREADS) void hist_kernel(const float *__restrict__ nH,
                                                            const float *__restrict__ qsrc,
                                                            int gamma, double csig,
                                                            uint32_t ncell, int nbx, int nby,
                                                            const double *__restrict__ edges,
                                                            float lox, float inv_wx, float loy,
                                                            float inv_wy, int vec,
                                                            unsigned long long *__restrict__ counts,
                                                            unsigned long long *__restrict__ limbs)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    double *se = reinterpret_cast<double *>(lds);                 // nbx + nby + 2
    unsigned long long *sacc =
        reinterpret_cast<unsigned long long *>(se + (nbx + nby + 2));   // nbx * HSLOT
    unsigned *scnt = reinterpret_cast<unsigned *>(sacc + size_t(nbx) * HSLOT);   // nbx * nby
    const int nbin = nbx * nby;
    for (int i = threadIdx.x; i < nbx + nby + 2; i += HIST_THREADS) se[i] = edges[i];
    for (int i = threadIdx.x; i < nbx * HSLOT; i += HIST_THREADS) sacc[i] = 0ull;
    for (int i = threadIdx.x; i < nbin; i += HIST_THREADS) scnt[i] = 0u;
    __syncthreads();
    const double *ex = se, *ey = se + nbx + 1;
    const float L10 = 0.301029995664f;   // log10(2)
    auto bins = [&](float h, float v, int &b, int &bx) {
        const double q = gamma ? csig * double(v) : double(v);
        bx = find_bin(double(h), L10 * flog2(h), ex, nbx, lox, inv_wx);
        const int by = find_bin(q, L10 * flog2(float(q)), ey, nby, loy, inv_wy);
        b = bx * nby + by;
    };
    // Eight consecutive cells per thread and iteration, read as two 16-byte
    // loads of each field (more loads in flight than one float per thread);
    // neighbouring cells that share a bin add their count once (runs).
    // 64-bit indices: ncell may approach 2^32.  The rest (and everything,
    // for unaligned fields) goes cell by cell.
    const uint64_t stride = uint64_t(gridDim.x) * HIST_THREADS;
    const uint64_t n8 = vec ? ncell / 8 : 0;
    const float4 *h4 = reinterpret_cast<const float4 *>(nH);
    const float4 *q4 = reinterpret_cast<const float4 *>(qsrc);
    for (uint64_t i = uint64_t(blockIdx.x) * HIST_THREADS + threadIdx.x; i < n8; i += stride) {
        const float4 ha = h4[2 * i], hb = h4[2 * i + 1];
        const float4 va = q4[2 * i], vb = q4[2 * i + 1];
        const float hh[8] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w};
        const float vv[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
        int b[8], bx[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) bins(hh[k], vv[k], b[k], bx[k]);
        unsigned run = 1;
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            if (b[k] == b[k - 1]) {
                ++run;
            } else {
                atomicAdd(&scnt[b[k - 1]], run);
                run = 1;
            }
        }
        atomicAdd(&scnt[b[7]], run);
        // exact sums: neighbouring cells of one density bin whose values
        // fall in the same limb are added in a register first
        int cb = -1, ck = 0;
        unsigned long long cp = 0ull;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int lk;
            unsigned long long p;
            if (!fixed_point(vv[k], lk, p)) {
                atomicAdd(&sacc[bx[k] * HSLOT + HLIMBS], 1ull);
                continue;
            }
            if (bx[k] == cb && lk == ck) {
                cp += p;
            } else {
                if (cb >= 0) limb_add(sacc + cb * HSLOT, ck, cp);
                cb = bx[k];
                ck = lk;
                cp = p;
            }
        }
        if (cb >= 0) limb_add(sacc + cb * HSLOT, ck, cp);
    }
    for (uint64_t i = n8 * 8 + uint64_t(blockIdx.x) * HIST_THREADS + threadIdx.x; i < ncell;
         i += stride) {
        int b, bx;
        bins(nH[i], qsrc[i], b, bx);
        atomicAdd(&scnt[b], 1u);
        int lk;
        unsigned long long p;
        if (fixed_point(qsrc[i], lk, p))
            limb_add(sacc + bx * HSLOT, lk, p);
        else
            atomicAdd(&sacc[bx * HSLOT + HLIMBS], 1ull);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbin; i += HIST_THREADS) {
        const unsigned c = scnt[i];
        if (c) atomicAdd(&counts[i], (unsigned long long)c);
    }
    for (int i = threadIdx.x; i < nbx * HSLOT; i += HIST_THREADS) {
        const unsigned long long v = sacc[i];
        if (v) atomicAdd(&limbs[i], v);
    }
}

// sums[i] = scale * (exact sum of bin i): the limbs' carries propagated into
// 32-bit digits, which are then added from the most significant down (a few
// ulp of FP64 at most; the same result on every run).
__global__ __launch_bounds__(256) void hist_sum_kernel(const unsigned long long *__restrict__ limbs,
                                                       int nbx, double scale,
                                                       double *__restrict__ sums)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nbx) return;
    const unsigned long long *a = limbs + size_t(i) * HSLOT;
    if (a[HLIMBS]) {
        sums[i] = __builtin_nan("");
        return;
    }
    uint32_t d[HLIMBS + 1];
    unsigned long long carry = 0;
#pragma unroll
    for (int k = 0; k < HLIMBS; ++k) {
        const unsigned long long t = a[k] + carry;   // a[k] <= (2^32 - 1)^2: no overflow
        d[k] = uint32_t(t);
        carry = t >> 32;
    }
    d[HLIMBS] = uint32_t(carry);
    double v = 0.0;
#pragma unroll
    for (int k = HLIMBS; k >= 0; --k) v += ldexp(double(d[k]), 32 * k - 149);
    sums[i] = v * scale;
}

size_t hist_lds_bytes(int nbx, int nby)
{
    return size_t(nbx + nby + 2) * 8 + size_t(nbx) * HSLOT * 8 + size_t(nbx) * nby * 4;
}

size_t hist_limb_count(int nbx) { return size_t(nbx) * HSLOT; }

int hist_blocks(uint32_t ncell)
{
    const uint64_t work = (uint64_t(ncell) + 7u) / 8u;
    const uint64_t want = (work + HIST_THREADS - 1) / HIST_THREADS;
    return int(want < 1 ? 1 : (want > HIST_MAX_BLOCKS ? HIST_MAX_BLOCKS : want));
}

hipError_t launch_hist(const float *nH, const float *q, int gamma, double csig, uint32_t ncell,
                       int nbx, int nby, const double *edges, float lox, float inv_wx,
                       float loy, float inv_wy, unsigned long long *counts,
                       unsigned long long *limbs, double *sums, hipStream_t s)
{
    const int vec = (reinterpret_cast<uintptr_t>(nH) % 16 == 0) &&
                    (reinterpret_cast<uintptr_t>(q) % 16 == 0);
    const int blocks = hist_blocks(ncell);
    hipLaunchKernelGGL(hist_kernel, dim3(blocks), dim3(HIST_THREADS), hist_lds_bytes(nbx, nby), s,
                       nH, q, gamma, csig, ncell, nbx, nby, edges, lox, inv_wx, loy, inv_wy, vec,
                       counts, limbs);
    hipLaunchKernelGGL(hist_sum_kernel, dim3((nbx + 255) / 256), dim3(256), 0, s,
                       static_cast<const unsigned long long *>(limbs), nbx, gamma ? csig : 1.0,
                       sums);
    return hipGetLastError();
}

// ------------------------------------------------ photoionisation plateau
// Mean of c sigma_n N over the cells with nH < nH_max (FP64): per-block
// partial sums and counts in a fixed order, then one block adds them.
constexpr int PLAT_THREADS = 256;

__global__ __launch_bounds__(PLAT_THREADS) void plateau_kernel(const float *__restrict__ nH,
                                                               const float *__restrict__ N,
                                                               uint32_t ncell, double nh_max,
                                                               double csig,
                                                               double *__restrict__ part)
{
    __shared__ double s[2][PLAT_THREADS / 64];
    double sum = 0.0, cnt = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * PLAT_THREADS;
    for (uint64_t i = uint64_t(blockIdx.x) * PLAT_THREADS + threadIdx.x; i < ncell; i += stride) {
        if (double(nH[i]) < nh_max) {
            sum += csig * double(N[i]);
            cnt += 1.0;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        cnt += __shfl_xor(cnt, off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s[0][wave] = sum;
        s[1][wave] = cnt;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < PLAT_THREADS / 64; ++w) v += s[threadIdx.x][w];
        part[size_t(blockIdx.x) * 2 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(64) void plateau_final_kernel(const double *__restrict__ part,
                                                           int nblocks, double *__restrict__ out)
{
    const int t = threadIdx.x;
    double sum = 0.0, cnt = 0.0;
    for (int b = t; b < nblocks; b += 64) {
        sum += part[size_t(b) * 2];
        cnt += part[size_t(b) * 2 + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        cnt += __shfl_xor(cnt, off);
    }
    if (t == 0) {
        out[0] = sum;
        out[1] = cnt;
    }
}

int plateau_blocks(uint32_t ncell)
{
    const uint64_t want = (uint64_t(ncell) + PLAT_THREADS * 16 - 1) / (PLAT_THREADS * 16);
    return int(want < 1 ? 1 : (want > 2048 ? 2048 : want));
}

hipError_t launch_plateau(const float *nH, const float *N, uint32_t ncell, double nh_max,
                          double csig, double *part, double *out, hipStream_t s)
{
    const int nb = plateau_blocks(ncell);
    hipLaunchKernelGGL(plateau_kernel, dim3(nb), dim3(PLAT_THREADS), 0, s, nH, N, ncell, nh_max,
                       csig, part);
    hipLaunchKernelGGL(plateau_final_kernel, dim3(1), dim3(64), 0, s,
                       static_cast<const double *>(part), nb, out);
    return hipGetLastError();
}

// Equilibrium neutral fraction y of the chemistry at fixed T and rate:
// C_R alpha nH (1-y)^2 = C_I Gamma y + beta nH (1-y) y, i.e. with
// a = C_R alpha nH, b = beta nH, g = C_I Gamma,
//   (a + b) y^2 - (2a + g + b) y + a = 0.
// The root in [0, 1] is taken as a over the larger root's numerator,
//   y = 2a / ((2a + g + b) + sqrt((g + b)^2 + 4 a g)),
// where every term is non-negative: no cancellation at either end (y << 1
// in ionised gas, 1 - y << 1 in shielded gas).  alpha and beta are the rate
// fits of the step's chemistry, evaluated in FP64 like the rest.
__global__ __launch_bounds__(256) void equilibrium_kernel(
    int64_t n, const double *__restrict__ nH, const double *__restrict__ T,
    double *__restrict__ xhi, int model, double gamma0, double inv_nstar, int clump,
    double cr_norm, double cr_exp, double ci_norm, double ci_exp)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const double nh = nH[i], t = T[i];
    if (!(nh > 0.0) || !isfinite(nh) || !(t >= 1.0) || !(t <= 1e9)) {
        xhi[i] = __builtin_nan("");
        return;
    }
    double g = gamma0;
    if (model == RT_JMODEL_EXP1) {
        g = gamma0 * exp(-nh * inv_nstar);
    } else if (model == RT_JMODEL_EXP4) {
        const double r = nh * inv_nstar, r2 = r * r;
        g = gamma0 * exp(-(r2 * r2));
    }
    double cR = 1.0, cI = 1.0;
    if (clump) {
        cR = fmax(1.0, cr_norm * pow(nh, cr_exp));
        cI = ci_norm * pow(nh, ci_exp);
    }
    const RateSetT<double> rs = rates_f64(t, 1.0);
    const double a = cR * rs.alpha * nh;
    const double b = rs.beta * nh;
    const double gi = cI * g;
    const double s = gi + b;
    const double den = (2.0 * a + s) + sqrt(s * s + 4.0 * a * gi);
    xhi[i] = den > 0.0 ? 2.0 * a / den : 1.0;
}

hipError_t launch_equilibrium(int64_t n, const double *nH, const double *T, double *xhi,
                              int model, double gamma0, double n_star, const rt_params &p,
                              hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    const double inv_ns = model == RT_JMODEL_UNIFORM ? 0.0 : 1.0 / n_star;
    hipLaunchKernelGGL(equilibrium_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, n, nH, T,
                       xhi, model, gamma0, inv_ns, p.clump, p.clump_cr_norm, p.clump_cr_exp,
                       p.clump_ci_norm, p.clump_ci_exp);
    return hipGetLastError();
}

}  // namespace rtk
