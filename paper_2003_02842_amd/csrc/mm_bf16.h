// BF16 rounding shared by the contraction's split step and the split fused into
// the FFT's row pass (device code only), so both round the same way.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

// Round to the nearest BF16, ties to even (the bits of the upper half).
__device__ __forceinline__ uint16_t bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// (x, y) times s, split into BF16 hi and lo parts packed as (x, y) pairs.  The
// product and the residual are rounded explicitly, so no caller's compilation can
// fuse them into one FMA and every caller produces the same bits.
__device__ __forceinline__ void bf16_split_pair(float x, float y, float s, uint32_t& hi, uint32_t& lo)
{
    const float vx = __fmul_rn(x, s), vy = __fmul_rn(y, s);
    const uint16_t h0 = bf16_rne(vx), h1 = bf16_rne(vy);
    const uint16_t l0 = bf16_rne(__fsub_rn(vx, bf16_to_f(h0))), l1 = bf16_rne(__fsub_rn(vy, bf16_to_f(h1)));
    hi = (uint32_t)h0 | ((uint32_t)h1 << 16);
    lo = (uint32_t)l0 | ((uint32_t)l1 << 16);
}

}  // namespace mm
