// Sources from stellar particles on gfx950 (Sec. 2.3): per particle, the
// nearest-grid-point cell and the effective emission rate over a snapshot
// interval.  One thread per particle, FP64 throughout, in the order
//   Ndot = ((Q m) / m_b) / L,
//   rate = ((Ndot (overlap / Delta)) f_esc) B,
// with overlap = max(0, min(a_next, L) - max(a_next - Delta, 0)), the time
// the particle's emitting ages [0, L] share with the interval.  No
// contraction into fused multiply-adds, so every product and quotient is
// one correctly rounded IEEE operation.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rt_internal.h"

namespace rtk {

constexpr double M_BARYON = 1.67262192e-24;  // g (proton mass)

__device__ __forceinline__ int32_t wrap_cell(double x, double dx, int n)
{
    const int64_t i = int64_t(floor(x / dx));
    int64_t r = i % n;
    if (r < 0) r += n;
    return int32_t(r);
}

__global__ __launch_bounds__(256) void particle_rate_kernel(
    int64_t n, const double *__restrict__ pos, const double *__restrict__ age_next,
    const double *__restrict__ lifetime, const double *__restrict__ q,
    const double *__restrict__ mass, double delta, double f_esc, double boost, double dx,
    int nx, int ny, int nz, int32_t *__restrict__ ijk, double *__restrict__ rate,
    int32_t *__restrict__ bad)
{
#pragma clang fp contract(off)
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= n) return;
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const double a = age_next[i], L = lifetime[i], Q = q[i], m = mass[i];
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(a) && L > 0.0 &&
                    isfinite(L) && Q >= 0.0 && isfinite(Q) && m >= 0.0 && isfinite(m);
    if (!ok) {
        bad[0] = 1;   // every writer stores the same value
        ijk[3 * i] = ijk[3 * i + 1] = ijk[3 * i + 2] = 0;
        rate[i] = 0.0;
        return;
    }
    ijk[3 * i] = wrap_cell(x, dx, nx);
    ijk[3 * i + 1] = wrap_cell(y, dx, ny);
    ijk[3 * i + 2] = wrap_cell(z, dx, nz);
    const double overlap = fmax(0.0, fmin(a, L) - fmax(a - delta, 0.0));
    const double Ndot = ((Q * m) / M_BARYON) / L;
    rate[i] = ((Ndot * (overlap / delta)) * f_esc) * boost;
}

hipError_t launch_particle_rates(int64_t n, const double *pos, const double *age_next,
                                 const double *lifetime, const double *q, const double *mass,
                                 double delta, double f_esc, double boost, double dx, int nx,
                                 int ny, int nz, int32_t *ijk, double *rate, int32_t *bad,
                                 hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(particle_rate_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, n, pos,
                       age_next, lifetime, q, mass, delta, f_esc, boost, dx, nx, ny, nz, ijk,
                       rate, bad);
    return hipGetLastError();
}

}  // namespace rtk
