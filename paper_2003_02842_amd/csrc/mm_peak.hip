// Measurement probe, not part of the estimator: the BF16 MFMA issue rate of
// gfx950 with no memory traffic (v_mfma_f32_32x32x16_bf16 back to back on
// independent accumulators), the achievable ceiling against which the
// contraction's SYRK kernel is judged beside the datasheet peak.  Built into
// its own library (libmm_peak.so); bench.py calls it.
#include <hip/hip_runtime.h>

#include <cstdint>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int kChains = 8;   // independent accumulators per wave

__global__ __launch_bounds__(256) void k_mfma_loop(int iters, float seed, float* __restrict__ out)
{
    bf16x8 a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(seed * (float)((int)threadIdx.x + i));
        b[i] = (__bf16)(seed * (float)(i + 1));
    }
    f32x16 acc[kChains];
    for (int c = 0; c < kChains; ++c)
        for (int i = 0; i < 16; ++i) acc[c][i] = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
    for (int c = 0; c < kChains; ++c)
        for (int i = 0; i < 16; ++i) s += acc[c][i];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// blocks workgroups of 256 threads, each wave issuing iters x 8 MFMAs of
// 32 x 32 x 16 (32768 flops each); out: blocks x 256 floats (device).
// Returns the hipError_t of the launch.
extern "C" int mm_peak_mfma_bf16(int blocks, int iters, float* out, void* stream)
{
    if (blocks <= 0 || iters <= 0 || !out) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mfma_loop, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, 1e-3f, out);
    return (int)hipGetLastError();
}
