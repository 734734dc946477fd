// Calibration kernels: the VALU and HBM rates this GPU actually sustains,
// the denominators of the measured-peak roofline fractions.
#include "kernels.h"

namespace gs {

// Eight independent FMA chains per lane: iters * 8 FMA instructions, no
// dependence stalls once a few waves share each SIMD.
__global__ __launch_bounds__(256) void k_probe_fma(float *__restrict__ out, int iters, float a,
                                                   float b)
{
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = (float)(threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i];
    if (s == 12345.0f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the chains live
}

// Eight independent chains of v_exp_f32.
__global__ __launch_bounds__(256) void k_probe_exp(float *__restrict__ out, int iters)
{
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = -0.001f * (float)(threadIdx.x + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = -__builtin_amdgcn_exp2f(x[i]);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i];
    if (s == 12345.0f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Plain device copy, 16 bytes per lane per step.
__global__ __launch_bounds__(256) void k_probe_copy(const float4 *__restrict__ src,
                                                    float4 *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

void launch_probe(int kind, float *scratch, int64_t n, int iters, const float4 *src, float4 *dst,
                  int blocks, hipStream_t st)
{
    if (kind == 0)
        hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, scratch, iters, 0.999f,
                           0.001f);
    else if (kind == 1)
        hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(256), 0, st, scratch, iters);
    else
        hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, st, src, dst, n);
}

}  // namespace gs
