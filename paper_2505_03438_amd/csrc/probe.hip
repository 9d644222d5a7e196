// Measurement probe (not part of the MD path): a dependent-FMA kernel that
// sustains the FP32 vector rate of the device as this library is compiled
// (packed FP32 instructions disabled), so that the force kernels' roofline
// can be quoted beside a measured ceiling as well as the published one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mdprobe.h"

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_fma_f32(int32_t iters, float b, float c, float *__restrict__ out)
{
    float a[kChains];
    for (int k = 0; k < kChains; k++) a[k] = (float)(threadIdx.x + k) * 1e-3f;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int k = 0; k < kChains; k++) a[k] = __builtin_fmaf(a[k], b, c);
    }
    float s = 0.f;
    for (int k = 0; k < kChains; k++) s += a[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int mdprobe_fma_f32(int32_t workgroups, int32_t iters, float *out, void *stream)
{
    if (workgroups <= 0 || iters <= 0 || !out) return -1;
    k_fma_f32<<<workgroups, 256, 0, (hipStream_t)stream>>>(iters, 0.999999f, 1e-7f, out);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" int64_t mdprobe_fma_f32_flops(int32_t workgroups, int32_t iters)
{
    return (int64_t)workgroups * 256 * (int64_t)iters * kChains * 2;
}
