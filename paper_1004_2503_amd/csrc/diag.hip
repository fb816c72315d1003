// Run diagnostics on gfx950: the distribution of cells over density and
// neutral fraction or photoionisation rate (Sec. 3.1.5), with the per-density
// bin sums that give the mean curves.
//
// Also the equilibrium neutral fraction under the self-shielding intensity
// models of the same section (one thread per element, FP64).
//
// One streaming pass over nH and the chosen quantity (8 bytes per cell).
// Each block keeps a private histogram in LDS (integer atomics) and FP64
// per-density-bin sums; blocks then add their non-zero bins to the global
// result (up to 8192 blocks: the LDS atomics need many waves in flight).  Bin decisions are exact: an FP32 logarithm proposes the bin and
// comparisons against the FP64 edges settle it.

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

__global__ __launch_bounds__(256) void hist_kernel(const float *__restrict__ nH,
                                                   const float *__restrict__ qsrc, int gamma,
                                                   double csig, uint32_t ncell, int nbx,
                                                   int nby, const double *__restrict__ edges,
                                                   float lox, float inv_wx, float loy,
                                                   float inv_wy, int vec,
                                                   unsigned long long *__restrict__ counts,
                                                   double *__restrict__ sums)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    double *se = reinterpret_cast<double *>(lds);                 // nbx + nby + 2
    double *ssum = se + (nbx + nby + 2);                          // nbx
    unsigned *scnt = reinterpret_cast<unsigned *>(ssum + nbx);    // nbx * nby
    const int nbin = nbx * nby;
    for (int i = threadIdx.x; i < nbx + nby + 2; i += 256) se[i] = edges[i];
    for (int i = threadIdx.x; i < nbx; i += 256) ssum[i] = 0.0;
    for (int i = threadIdx.x; i < nbin; i += 256) scnt[i] = 0u;
    __syncthreads();
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
    // neighbouring cells that share a bin are combined before the LDS
    // atomics, which bound the kernel.  64-bit indices: ncell may approach
    // 2^32.  The rest (and everything, for unaligned fields) goes cell by
    // cell.
    const uint64_t stride = uint64_t(gridDim.x) * 256u;
    const uint64_t n8 = vec ? ncell / 8 : 0;
    const float4 *h4 = reinterpret_cast<const float4 *>(nH);
    const float4 *q4 = reinterpret_cast<const float4 *>(qsrc);
    for (uint64_t i = uint64_t(blockIdx.x) * 256u + threadIdx.x; i < n8; i += stride) {
        const float4 ha = h4[2 * i], hb = h4[2 * i + 1];
        const float4 va = q4[2 * i], vb = q4[2 * i + 1];
        const float hh[8] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w};
        const float vv[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
        int b[8], bx[8];
        double q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) bins(hh[k], vv[k], b[k], bx[k], q[k]);
        unsigned run = 1;
        double qs = q[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            if (b[k] == b[k - 1]) {
                ++run;
            } else {
                atomicAdd(&scnt[b[k - 1]], run);
                run = 1;
            }
            if (bx[k] == bx[k - 1]) {
                qs += q[k];
            } else {
                atomicAdd(&ssum[bx[k - 1]], qs);
                qs = q[k];
            }
        }
        atomicAdd(&scnt[b[7]], run);
        atomicAdd(&ssum[bx[7]], qs);
    }
    for (uint64_t i = n8 * 8 + uint64_t(blockIdx.x) * 256u + threadIdx.x; i < ncell;
         i += stride) {
        int b, bx;
        double q;
        bins(nH[i], qsrc[i], b, bx, q);
        atomicAdd(&scnt[b], 1u);
        atomicAdd(&ssum[bx], q);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbin; i += 256) {
        const unsigned c = scnt[i];
        if (c) atomicAdd(&counts[i], (unsigned long long)c);
    }
    for (int i = threadIdx.x; i < nbx; i += 256) {
        const double v = ssum[i];
        if (v != 0.0) atomicAdd(&sums[i], v);
    }
}

size_t hist_lds_bytes(int nbx, int nby)
{
    return size_t(nbx + nby + 2) * 8 + size_t(nbx) * 8 + size_t(nbx) * nby * 4;
}

hipError_t launch_hist(const float *nH, const float *q, int gamma, double csig, uint32_t ncell,
                       int nbx, int nby, const double *edges, float lox, float inv_wx,
                       float loy, float inv_wy, unsigned long long *counts, double *sums,
                       hipStream_t s)
{
    const int vec = (reinterpret_cast<uintptr_t>(nH) % 16 == 0) &&
                    (reinterpret_cast<uintptr_t>(q) % 16 == 0);
    const uint64_t work = vec ? (uint64_t(ncell) + 7u) / 8u : uint64_t(ncell);
    const uint64_t want = (work + 255u) / 256u;
    const unsigned blocks = want < 8192u ? (want > 0 ? unsigned(want) : 1u) : 8192u;
    hipLaunchKernelGGL(hist_kernel, dim3(blocks), dim3(256), hist_lds_bytes(nbx, nby), s, nH,
                       q, gamma, csig, ncell, nbx, nby, edges, lox, inv_wx, loy, inv_wy, vec,
                       counts, sums);
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
