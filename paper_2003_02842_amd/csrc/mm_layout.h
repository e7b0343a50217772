// LDS layouts of the spreading and fused NUFFT kernels, as sizes the host planner
// needs too (no device code, so the planner builds as plain host C++).
#pragma once
#include <stddef.h>

#include "mm_internal.h"

// Events staged per LDS chunk (a multiple of 256).
#ifndef MM_POLY_CHUNK
#define MM_POLY_CHUNK 512
#endif

namespace mm {

constexpr int kFusedThreads = 512;                                 // eight waves per series
constexpr int kFusedPPT = kFusedMaxCells / (2 * kFusedThreads);    // cell pairs per thread
constexpr int kFusedEV = 2;                                        // events per thread per staged chunk


template <int W, int PPT, int NT = 256, int EV = 0>
struct SpreadLds {
    static constexpr int TC = 2 * NT * PPT;             // cells of a tile
    static constexpr int M = (W + 2) & ~1;               // even ring, >= W + 1
    static constexpr int EC0 = (M <= 12 || MM_POLY_CHUNK <= 256) ? MM_POLY_CHUNK : MM_POLY_CHUNK / 2;   // ~25 KB
    // events per chunk, a multiple of NT: EV per thread if given, else about EC0
    static constexpr int EC = EV > 0 ? EV * NT : (EC0 < NT ? NT : EC0);
    static constexpr int ring_floats = EC * M;
    static constexpr int first_len = TC + W + 2;
    static constexpr size_t bytes = 4 * (size_t)ring_floats + 2 * (size_t)EC + 2 * (size_t)first_len;
};

// LDS layout of k_nufft_fused in float2 units: tables, then the grid z (also the
// row pass's output rows), then the exchange buffer sh.
struct FusedLds {
    int tw1, tw2, Llo, Lhi, Mlo, Mhi, z, sh, total;
};
__host__ __device__ inline FusedLds fused_lds(int L1, int L2, int A1, int B1, int lo_bits, int n_hi)
{
    FusedLds f;
    const int LO = 1 << lo_bits, P = L1 / 2 + 1, rs = L2 + 1;
    f.tw1 = 0;
    f.tw2 = f.tw1 + L1;
    f.Llo = f.tw2 + L2;
    f.Lhi = f.Llo + LO;
    f.Mlo = f.Lhi + n_hi;
    f.Mhi = f.Mlo + LO;
    f.z = (f.Mhi + n_hi + 1) & ~1;                       // 16-byte aligned
    const int zlen = L1 * L2 > 2 * P * rs ? L1 * L2 : 2 * P * rs;
    f.sh = f.z + ((zlen + 1) & ~1);
    f.total = f.sh + (A1 * (B1 * L2 + 1) > 2 * P * rs ? A1 * (B1 * L2 + 1) : 2 * P * rs);
    return f;
}

}  // namespace mm
