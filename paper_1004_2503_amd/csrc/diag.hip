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
// result.  Bin decisions are exact: an FP32 logarithm proposes the bin and
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
                                                   float inv_wy,
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
    // 64-bit index: ncell may approach 2^32, where a 32-bit stride would wrap
    const uint64_t stride = uint64_t(gridDim.x) * 256u;
    for (uint64_t i = uint64_t(blockIdx.x) * 256u + threadIdx.x; i < ncell; i += stride) {
        const float h = nH[i];
        const float s = qsrc[i];
        const double q = gamma ? csig * double(s) : double(s);
        const int bx = find_bin(double(h), L10 * flog2(h), ex, nbx, lox, inv_wx);
        const int by = find_bin(q, L10 * flog2(float(q)), ey, nby, loy, inv_wy);
        atomicAdd(&scnt[bx * nby + by], 1u);
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
    const uint32_t want = (ncell + 255u) / 256u;
    const unsigned blocks = want < 2048u ? (want > 0 ? want : 1u) : 2048u;
    hipLaunchKernelGGL(hist_kernel, dim3(blocks), dim3(256), hist_lds_bytes(nbx, nby), s, nH,
                       q, gamma, csig, ncell, nbx, nby, edges, lox, inv_wx, loy, inv_wy,
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
// in ionised gas, 1 - y << 1 in shielded gas).  alpha and beta are the FP32
// rate fits of the step's chemistry; the rest is FP64.
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
    const RateSet rs = rates_f32(float(t), 1.0f);
    const double a = cR * double(rs.alpha) * nh;
    const double b = double(rs.beta) * nh;
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
