// Measurement probes, not part of the estimator: the BF16 MFMA issue rate of
// gfx950 with no memory traffic (v_mfma_f32_32x32x16_bf16 back to back on
// independent accumulators) and a streaming copy, the achievable ceilings
// against which the contraction and the HBM-bound kernels are compared beside the
// datasheet peaks.  Built into their own library (libmm_peak.so); bench.py
// calls them.
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

// Streaming copy of n16 16-byte words: each thread moves four words per trip,
// all four loads issued before the stores, in a grid-stride loop.
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

// Copies n16 16-byte words from src to dst (device pointers, 16-byte aligned)
// with blocks workgroups of 256 threads.  Returns the hipError_t of the launch.
extern "C" int mm_peak_copy(const void* src, void* dst, int64_t n16, int blocks, void* stream)
{
    if (blocks <= 0 || n16 < 0 || !src || !dst || (((uintptr_t)src | (uintptr_t)dst) & 15)) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4*)src,
                       (float4*)dst, n16);
    return (int)hipGetLastError();
}

// blocks workgroups of 256 threads, each wave issuing iters x 8 MFMAs of
// 32 x 32 x 16 (32768 flops each); out: blocks x 256 floats (device).
// Returns the hipError_t of the launch.
extern "C" int mm_peak_mfma_bf16(int blocks, int iters, float* out, void* stream)
{
    if (blocks <= 0 || iters <= 0 || !out) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mfma_loop, dim3(blocks), dim3(256), 0, (hipStream_t)stream, iters, 1e-3f, out);
    return (int)hipGetLastError();
}
