// Run diagnostics on gfx950: the distribution of cells over density and
// neutral fraction or photoionisation rate (Sec. 3.1.5), with the per-density
// bin sums that give the mean curves.
//
// Also the equilibrium neutral fraction under the self-shielding intensity
// models of the same section (one thread per element, FP64).
//
// One streaming pass over nH and the chosen quantity (8 bytes per cell).
// Each block keeps a private histogram in LDS (integer atomics) and FP64
// per-density-bin sums (deterministic: see hist_kernel); blocks then add
// their non-zero count bins to the global result.  Bin decisions are exact:
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

// Sums of q per density bin are made deterministic: every wavefront adds
// into its own LDS row, and within a wavefront the lanes holding the same
// bin are summed by a fixed butterfly before one lane adds the result (a
// loop over the distinct bins present); the block then writes the sum of
// its rows, in wavefront order, as its partial row, and hist_sum_kernel
// adds the partial rows in block order.  Counts are integers, added with
// atomics (exact in any order).
constexpr int HIST_THREADS = 256, HIST_WAVES = HIST_THREADS / 64;

__device__ __forceinline__ void wave_bin_add(double *row, int bx, double q, bool active)
{
    const int lane = threadIdx.x & 63;
    unsigned long long pend = __ballot(active);
    while (pend) {
        const int leader = __builtin_ctzll(pend);
        const int b = __shfl(bx, leader);
        const bool mine = active && bx == b;
        const unsigned long long m = __ballot(mine);
        double v = mine ? q : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == leader) row[b] += v;
        pend &= ~m;
    }
}

__global__ __launch_bounds__(HIST_THREADS) void hist_kernel(const float *__restrict__ nH,
                                                            const float *__restrict__ qsrc,
                                                            int gamma, double csig,
                                                            uint32_t ncell, int nbx, int nby,
                                                            const double *__restrict__ edges,
                                                            float lox, float inv_wx, float loy,
                                                            float inv_wy, int vec,
                                                            unsigned long long *__restrict__ counts,
                                                            double *__restrict__ partials)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    double *se = reinterpret_cast<double *>(lds);                 // nbx + nby + 2
    double *ssum = se + (nbx + nby + 2);                          // HIST_WAVES rows of nbx
    unsigned *scnt = reinterpret_cast<unsigned *>(ssum + HIST_WAVES * nbx);   // nbx * nby
    const int nbin = nbx * nby;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < nbx + nby + 2; i += HIST_THREADS) se[i] = edges[i];
    for (int i = threadIdx.x; i < HIST_WAVES * nbx; i += HIST_THREADS) ssum[i] = 0.0;
    for (int i = threadIdx.x; i < nbin; i += HIST_THREADS) scnt[i] = 0u;
    __syncthreads();
    double *row = ssum + wave * nbx;
    const double *ex = se, *ey = se + nbx + 1;
    const float L10 = 0.301029995664f;   // log10(2)
    auto bins = [&](float h, float v, int &b, int &bx, double &q) {
        q = gamma ? csig * double(v) : double(v);
        bx = find_bin(double(h), L10 * flog2(h), ex, nbx, lox, inv_wx);
        const int by = find_bin(q, L10 * flog2(float(q)), ey, nby, loy, inv_wy);
        b = bx * nby + by;
    };
    // Eight consecutive cells per thread and iteration, read as two 16-byte
    // loads of each field (more loads in flight than one float per thread);
    // neighbouring cells that share a bin are combined first (runs).  The
    // loops run the same number of times on every lane of a wavefront (the
    // wavefront-wide sums need all lanes).  64-bit indices: ncell may
    // approach 2^32.  The rest (and everything, for unaligned fields) goes
    // cell by cell.
    const uint64_t stride = uint64_t(gridDim.x) * HIST_THREADS;
    const uint64_t n8 = vec ? ncell / 8 : 0;
    const float4 *h4 = reinterpret_cast<const float4 *>(nH);
    const float4 *q4 = reinterpret_cast<const float4 *>(qsrc);
    const uint64_t wbase = uint64_t(blockIdx.x) * HIST_THREADS + uint64_t(threadIdx.x & ~63);
    for (uint64_t i0 = wbase; i0 < n8; i0 += stride) {
        const uint64_t i = i0 + (threadIdx.x & 63);
        const bool in = i < n8;
        float hh[8], vv[8];
        if (in) {
            const float4 ha = h4[2 * i], hb = h4[2 * i + 1];
            const float4 va = q4[2 * i], vb = q4[2 * i + 1];
            hh[0] = ha.x; hh[1] = ha.y; hh[2] = ha.z; hh[3] = ha.w;
            hh[4] = hb.x; hh[5] = hb.y; hh[6] = hb.z; hh[7] = hb.w;
            vv[0] = va.x; vv[1] = va.y; vv[2] = va.z; vv[3] = va.w;
            vv[4] = vb.x; vv[5] = vb.y; vv[6] = vb.z; vv[7] = vb.w;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) hh[k] = vv[k] = 1.0f;
        }
        int b[8], bx[8];
        double q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) bins(hh[k], vv[k], b[k], bx[k], q[k]);
        if (in) {
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
        }
        // density-bin sums: runs of equal density bins within the thread,
        // each closed run added to the wavefront's row
        double qs = q[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            const bool close = bx[k] != bx[k - 1];
            wave_bin_add(row, bx[k - 1], qs, in && close);
            qs = close ? q[k] : qs + q[k];
        }
        wave_bin_add(row, bx[7], qs, in);
    }
    const uint64_t rest0 = n8 * 8;
    for (uint64_t i0 = rest0 + wbase; i0 < ncell; i0 += stride) {
        const uint64_t i = i0 + (threadIdx.x & 63);
        const bool in = i < ncell;
        int b = 0, bx = 0;
        double q = 0.0;
        if (in) {
            bins(nH[i], qsrc[i], b, bx, q);
            atomicAdd(&scnt[b], 1u);
        }
        wave_bin_add(row, bx, q, in);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbin; i += HIST_THREADS) {
        const unsigned c = scnt[i];
        if (c) atomicAdd(&counts[i], (unsigned long long)c);
    }
    for (int i = threadIdx.x; i < nbx; i += HIST_THREADS) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < HIST_WAVES; ++w) v += ssum[w * nbx + i];
        partials[size_t(blockIdx.x) * nbx + i] = v;
    }
}

// sums[i] = the partial rows' bin i added in block order (one thread per bin).
__global__ __launch_bounds__(256) void hist_sum_kernel(const double *__restrict__ partials,
                                                       int nblocks, int nbx,
                                                       double *__restrict__ sums)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nbx) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partials[size_t(b) * nbx + i];
    sums[i] = v;
}

size_t hist_lds_bytes(int nbx, int nby)
{
    return size_t(nbx + nby + 2) * 8 + size_t(HIST_WAVES) * nbx * 8 + size_t(nbx) * nby * 4;
}

int hist_blocks(uint32_t ncell)
{
    const uint64_t work = (uint64_t(ncell) + 7u) / 8u;
    const uint64_t want = (work + HIST_THREADS - 1) / HIST_THREADS;
    return int(want < 1 ? 1 : (want > HIST_MAX_BLOCKS ? HIST_MAX_BLOCKS : want));
}

hipError_t launch_hist(const float *nH, const float *q, int gamma, double csig, uint32_t ncell,
                       int nbx, int nby, const double *edges, float lox, float inv_wx,
                       float loy, float inv_wy, unsigned long long *counts, double *partials,
                       double *sums, hipStream_t s)
{
    const int vec = (reinterpret_cast<uintptr_t>(nH) % 16 == 0) &&
                    (reinterpret_cast<uintptr_t>(q) % 16 == 0);
    const int blocks = hist_blocks(ncell);
    hipLaunchKernelGGL(hist_kernel, dim3(blocks), dim3(HIST_THREADS), hist_lds_bytes(nbx, nby), s,
                       nH, q, gamma, csig, ncell, nbx, nby, edges, lox, inv_wx, loy, inv_wy, vec,
                       counts, partials);
    hipLaunchKernelGGL(hist_sum_kernel, dim3((nbx + 255) / 256), dim3(256), 0, s,
                       static_cast<const double *>(partials), blocks, nbx, sums);
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
