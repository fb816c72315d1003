// The achievable HBM bandwidth of the step kernel's stream mix: a plain
// grid-stride kernel that reads nin arrays and writes nout arrays of n
// floats (each output the sum of all inputs, so that no read can be
// skipped), with non-temporal stores as in the step, and the same 7-read /
// 6-write mix in the step's tile-marching order.  They measure the ceiling
// the step's pattern can reach on the device; they are not part of the
// method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_internal.h"

namespace rtk {

constexpr int PROBE_MAX = 16;
struct ProbePtrs {
    const float *in[PROBE_MAX];
    float *out[PROBE_MAX];
};

__global__ __launch_bounds__(256) void stream_probe_kernel(ProbePtrs p, int nin, int nout,
                                                           uint64_t n)
{
    const uint64_t stride = uint64_t(gridDim.x) * 256u;
    for (uint64_t i = uint64_t(blockIdx.x) * 256u + threadIdx.x; i < n; i += stride) {
        float v[PROBE_MAX];
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < PROBE_MAX; ++k) {
            v[k] = k < nin ? p.in[k][i] : 0.0f;
            s += v[k];
        }
#pragma unroll
        for (int k = 0; k < PROBE_MAX; ++k)
            if (k < nout) __builtin_nontemporal_store(s + v[k], &p.out[k][i]);
    }
}

// The same mix in the LF step kernel's own access pattern: 64 x 16 tiles
// of 1024 threads march 128 planes in z with the next plane's seven loads in
// flight, one barrier per plane and 96 KiB of LDS per block, so that one
// block runs per compute unit as in the step; no stencil, halo, sources or
// chemistry.  Each output is the plane's sum of the inputs plus one value
// from another wavefront (through LDS, double-buffered by plane parity).
constexpr int MP_TX = 64, MP_TY = 16, MP_ZC = 128, MP_NIN = 7, MP_NOUT = 6;
constexpr int MP_LDS = 96 * 1024;

__global__ __launch_bounds__(MP_TX *MP_TY) void march_probe_kernel(ProbePtrs p, int nx, int ny)
{
    extern __shared__ float mp_lds[];
    const int tid = threadIdx.x;
    const uint64_t x = uint64_t(blockIdx.x) * MP_TX + (tid & 63);
    const uint64_t y = uint64_t(blockIdx.y) * MP_TY + (tid >> 6);
    const int z0 = blockIdx.z * MP_ZC;
    const uint64_t plane = uint64_t(nx) * uint64_t(ny), col = y * uint64_t(nx) + x;
    float r[MP_NIN];
#pragma unroll
    for (int k = 0; k < MP_NIN; ++k) r[k] = p.in[k][col + uint64_t(z0) * plane];
    for (int z = z0; z < z0 + MP_ZC; ++z) {
        float v[MP_NIN];
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < MP_NIN; ++k) {
            v[k] = r[k];
            s += v[k];
        }
        const uint64_t zn = uint64_t(min(z + 1, z0 + MP_ZC - 1));
#pragma unroll
        for (int k = 0; k < MP_NIN; ++k) r[k] = p.in[k][col + zn * plane];
        float *buf = mp_lds + (z & 1) * (MP_TX * MP_TY);
        buf[tid] = s;
        __syncthreads();
        s += buf[(tid + 64) & (MP_TX * MP_TY - 1)];
#pragma unroll
        for (int k = 0; k < MP_NOUT; ++k)
            __builtin_nontemporal_store(s + v[k], &p.out[k][col + uint64_t(z) * plane]);
    }
}

}  // namespace rtk

using namespace rtk;

namespace {

// one warm-up launch, then reps timed launches with HIP events on s
template <typename Launch>
int time_launches(hipStream_t s, int reps, double *ms, Launch launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return RT_E_HIP;
    }
    int rc = RT_OK;
    launch();
    if (hipEventRecord(a, s) != hipSuccess) rc = RT_E_HIP;
    for (int r = 0; r < reps && rc == RT_OK; ++r) launch();
    float t = 0.0f;
    if (rc == RT_OK && (hipGetLastError() != hipSuccess || hipEventRecord(b, s) != hipSuccess ||
                        hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&t, a, b) != hipSuccess))
        rc = RT_E_HIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc == RT_OK) *ms = double(t) / reps;
    return rc;
}

}  // namespace

extern "C" int rt_stream_probe(const float *const *in, int32_t nin, float *const *out,
                               int32_t nout, int64_t n, int32_t blocks, int32_t reps,
                               double *ms, void *hip_stream)
{
    if (!in || !out || !ms || nin < 1 || nin > PROBE_MAX || nout < 1 || nout > PROBE_MAX ||
        n < 1 || blocks < 1 || reps < 1)
        return RT_E_ARG;
    ProbePtrs p{};
    for (int k = 0; k < nin; ++k) {
        if (!in[k]) return RT_E_ARG;
        p.in[k] = in[k];
    }
    for (int k = 0; k < nout; ++k) {
        if (!out[k]) return RT_E_ARG;
        p.out[k] = out[k];
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    return time_launches(s, reps, ms, [&] {
        hipLaunchKernelGGL(stream_probe_kernel, dim3(blocks), dim3(256), 0, s, p, nin, nout,
                           uint64_t(n));
    });
}

extern "C" int rt_march_probe(const float *const *in, float *const *out, int32_t nx,
                              int32_t ny, int32_t nz, int32_t reps, double *ms,
                              void *hip_stream)
{
    if (!in || !out || !ms || reps < 1 || nx < MP_TX || ny < MP_TY || nz < MP_ZC ||
        nx % MP_TX || ny % MP_TY || nz % MP_ZC || ny / MP_TY > 65535 || nz / MP_ZC > 65535)
        return RT_E_ARG;
    ProbePtrs p{};
    for (int k = 0; k < MP_NIN; ++k) {
        if (!in[k]) return RT_E_ARG;
        p.in[k] = in[k];
    }
    for (int k = 0; k < MP_NOUT; ++k) {
        if (!out[k]) return RT_E_ARG;
        p.out[k] = out[k];
    }
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(march_probe_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, MP_LDS) != hipSuccess)
        return RT_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const dim3 grid(nx / MP_TX, ny / MP_TY, nz / MP_ZC);
    return time_launches(s, reps, ms, [&] {
        hipLaunchKernelGGL(march_probe_kernel, grid, dim3(MP_TX * MP_TY), MP_LDS, s, p, nx, ny);
    });
}
