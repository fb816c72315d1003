// The achievable HBM bandwidth of the step kernel's stream mix: a plain
// grid-stride kernel that reads nin arrays and writes nout arrays of n
// floats (each output the sum of all inputs, so that no read can be
// skipped), with non-temporal stores as in the step.  It measures the
// ceiling the step's 7-read / 6-write pattern can reach on the device; it
// is not part of the method.
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

}  // namespace rtk

using namespace rtk;

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
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return RT_E_HIP;
    }
    int rc = RT_OK;
    hipLaunchKernelGGL(stream_probe_kernel, dim3(blocks), dim3(256), 0, s, p, nin, nout,
                       uint64_t(n));   // warm-up
    if (hipEventRecord(a, s) != hipSuccess) rc = RT_E_HIP;
    for (int r = 0; r < reps && rc == RT_OK; ++r)
        hipLaunchKernelGGL(stream_probe_kernel, dim3(blocks), dim3(256), 0, s, p, nin, nout,
                           uint64_t(n));
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
