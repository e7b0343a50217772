// Fused type-1 NUFFT of small grids (Sec. 2.2.5, Eqs. Der:15-17): one workgroup
// of 512 threads per series keeps the whole oversampled grid (Mr <= 8192 cells)
// in LDS.
//
//   k_nufft_fused  1. spreading of the series' events (spread_tile_poly, one tile
//                     covering the whole grid, the three wrap ranges of the tile
//                     search), the grid left in registers;
//                  2. the grid, as the packed complex sequence z_j = x_2j + i x_2j+1
//                     of length L = Mr/2 viewed as L1 x L2, written into LDS;
//                  3. the column pass (length-L1 transforms of the L2 columns in two
//                     register-codelet steps through LDS, times W_L^{k1 l2}) in
//                     place;
//                  4. the row pass (length-L2 transforms of the rows k1 and L1 - k1
//                     in two steps), then the real-input untangling, the
//                     deconvolution (Eq. Der:17) and the 1/2pi, writing c_k,
//                     k = 0..N, to HBM.
// Only the events are read and only the coefficients written; the grid never
// reaches HBM.  The LDS holds the FFT tables, the grid and one exchange buffer;
// the spreading's rings, keys and cell index sit over the latter two while they
// are not yet in use.
#include <hip/hip_runtime.h>

#include "mm_fft_codelets.h"
#include "mm_internal.h"
#include "mm_layout.h"
#include "mm_spread.h"

namespace mm {

// Codelet sizes of the fused kernel's FFT steps: up to 16 points, which keeps the
// register arrays of a step (and so the kernel's VGPRs) small.
#define MM_CODELETS16(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16)

template <int W>
__global__ __launch_bounds__(kFusedThreads) void k_nufft_fused(const double* __restrict__ t, DpAny dp,
                                                     double t0, double scale, int Mr, double hw, PolyParams pp,
                                                     const int64_t* __restrict__ ranges, int L1, int L2, int A1,
                                                     int B1, int A2, int B2, const float2* __restrict__ tw1g,
                                                     const float2* __restrict__ tw2g, const float2* __restrict__ Llog,
                                                     const float2* __restrict__ Lhig, const float2* __restrict__ Mlog,
                                                     const float2* __restrict__ Mhig, int lo_bits, int n_hi,
                                                     const float* __restrict__ dfac, int N, float2* __restrict__ coef,
                                                     int64_t ldc)
{
    using C = float2;
    constexpr int NT = kFusedThreads;
    using SL = SpreadLds<W, kFusedPPT, NT, kFusedEV>;
    extern __shared__ __align__(16) char smem_raw[];
    C* const base = reinterpret_cast<C*>(smem_raw);
    const FusedLds lay = fused_lds(L1, L2, A1, B1, lo_bits, n_hi);
    C* const tw1 = base + lay.tw1;
    C* const tw2 = base + lay.tw2;
    C* const Llo = base + lay.Llo;
    C* const Lhi = base + lay.Lhi;
    C* const Mlo = base + lay.Mlo;
    C* const Mhi = base + lay.Mhi;
    C* const z = base + lay.z;
    C* const sh = base + lay.sh;
    const int tid = (int)threadIdx.x;
    const int LO = 1 << lo_bits;
    for (int i = tid; i < L1; i += NT) tw1[i] = tw1g[i];
    for (int i = tid; i < L2; i += NT) tw2[i] = tw2g[i];
    for (int i = tid; i < LO; i += NT) {
        Llo[i] = Llog[i];
        Mlo[i] = Mlog[i];
    }
    for (int i = tid; i < n_hi; i += NT) {
        Lhi[i] = Lhig[i];
        Mhi[i] = Mhig[i];
    }
    // 1. spreading: the rings, keys and cell index over z and sh
    const int s = blockIdx.x;
    float* const ring = reinterpret_cast<float*>(z);
    unsigned short* const keys = reinterpret_cast<unsigned short*>(ring + SL::ring_floats);
    unsigned short* const first = keys + SL::EC;
    float acc0[kFusedPPT], acc1[kFusedPPT];
    spread_tile_poly<DpAny, W, kFusedPPT, NT, kFusedEV>(t, dp, t0, scale, Mr, hw, pp, ranges + 6 * (int64_t)s, 0, Mr, ring, keys,
                                          first, acc0, acc1);
    __syncthreads();   // every gather is done: the grid goes over the rings
    // 2. cell pair (c, c+1), c = 2 (tid + NT r), is z_j with j = tid + NT r, at row j / L2,
    // column j % L2 of the unpadded L1 x L2 view, i.e. at z[j]
    const int L = Mr >> 1;
#pragma unroll
    for (int r = 0; r < kFusedPPT; ++r) {
        const int j = tid + NT * r;
        if (j < L) z[j] = make_float2(acc0[r], acc1[r]);
    }
    __syncthreads();
    // 3. column pass, all L2 columns: step A (tasks nb < B1) into sh, step B back into z
    const int blk = B1 * L2 + 1;
    for (int task = tid; task < B1 * L2; task += NT) {
        const int nb = task / L2, col = task - nb * L2;
        switch (A1) {
#define MM_CASE_A(n) case n: col_step_a<float, n>(z, L2, B1, nb, col, tw1, sh, blk, nb * L2 + col); break;
            MM_CODELETS16(MM_CASE_A)
#undef MM_CASE_A
        }
    }
    __syncthreads();
    for (int task = tid; task < A1 * L2; task += NT) {
        const int ka = task / L2, col = task - ka * L2;
        switch (B1) {
#define MM_CASE_B(n) case n: col_step_b<float, n>(z, L2, A1, ka, col, L2, sh, blk, col, Llo, Lhi, lo_bits); break;
            MM_CODELETS16(MM_CASE_B)
#undef MM_CASE_B
        }
    }
    __syncthreads();
    // 4. row pass: exchange row r of sh holds matrix row i = r/2 (r even) or its
    // mirror (L1 - i) mod L1 (r odd), i < P; step B writes the outputs, in natural
    // order, to the same rows of z (free once step A has read it)
    const int P = L1 / 2 + 1, rs = L2 + 1;
    for (int task = tid; task < 2 * P * B2; task += NT) {
        const int r = task / B2, nb = task - r * B2;
        const int i = r >> 1;
        const int k1 = (r & 1) ? (L1 - i) % L1 : i;
        switch (A2) {
#define MM_CASE_A(n) case n: row_step_a<float, n>(z + k1 * L2, B2, nb, tw2, sh + r * rs); break;
            MM_CODELETS16(MM_CASE_A)
#undef MM_CASE_A
        }
    }
    __syncthreads();
    for (int task = tid; task < 2 * P * A2; task += NT) {
        const int r = task / A2, ka = task - r * A2;
        C y[16];
        switch (B2) {
#define MM_CASE_B(n)                                         \
    case n:                                                  \
        row_step_b<float, n>(sh + r * rs, ka, y);            \
        row_store_b<float, n>(z + r * rs, A2, ka, y);        \
        break;
            MM_CODELETS16(MM_CASE_B)
#undef MM_CASE_B
        }
    }
    __syncthreads();
    // X_k = (Z_k + conj Z_{L-k})/2 - (i/2) W_Mr^k (Z_k - conj Z_{L-k}), k = k1 + L1 k2 <= N:
    // Z_k in the row of k1, Z_{L-k} in the mirror row at column L2-1-k2, or (L2-k2) mod L2
    // when k1 = 0; then the deconvolution factor (with 1/2pi)
    C* const out = coef + (int64_t)s * ldc;
    for (int k = tid; k <= N; k += NT) {
        const int k2 = k / L1, k1 = k - k2 * L1;
        const bool low = 2 * k1 <= L1;
        const int i = low ? k1 : L1 - k1, side = low ? 0 : 1;
        const int k2m = (k1 == 0) ? (k2 == 0 ? 0 : L2 - k2) : (L2 - 1 - k2);
        const C Zk = z[(2 * i + side) * rs + k2];
        const C Zm = z[(2 * i + 1 - side) * rs + k2m];
        const C Av = C{Zk.x + Zm.x, Zk.y - Zm.y};
        const C Bv = C{Zk.x - Zm.x, Zk.y + Zm.y};
        const C WB = cmulf(tw_split(Mlo, Mhi, k, lo_bits), Bv);
        const float d = dfac[k] * 0.5f;
        out[k] = C{(Av.x + WB.y) * d, (Av.y - WB.x) * d};
    }
}

// Bytes of the spreading's rings, keys and cell index for a plan's width.
template <int W>
static void fused_w(const Plan& p, const NufftWs& w, char* ws, int32_t S, const double* t, DpAny dp,
                    double t0, double scale, const int64_t* ranges, float2* coef, int64_t ldc, hipStream_t st)
{
    static_assert(SpreadLds<W, kFusedPPT, kFusedThreads, kFusedEV>::TC == kFusedMaxCells, "one tile covers the grid");
    hipLaunchKernelGGL(k_nufft_fused<W>, dim3(S), dim3(kFusedThreads), fused_lds_bytes(p), st, t, dp, t0, scale, p.Mr, p.kp.hw,
                       p.pp, ranges, p.L1, p.L2, p.A1, p.B1, p.A2, p.B2, (const float2*)(ws + w.tw1),
                       (const float2*)(ws + w.tw2), (const float2*)(ws + w.tLlo), (const float2*)(ws + w.tLhi),
                       (const float2*)(ws + w.tMlo), (const float2*)(ws + w.tMhi), p.tw_lo_bits, p.tw_hi_L,
                       (const float*)(ws + w.dfac), p.N, coef, ldc);
}

hipError_t launch_nufft_fused(const Plan& p, const NufftWs& w, char* ws, int32_t S, const double* t, const void* dp,
                              int dp_fp64, double t0, double T, void* coef, int64_t ldc, hipStream_t st)
{
    if (S <= 0) return hipSuccess;
    const double scale = (double)p.Mr / (T - t0);
    const int64_t* ranges = (const int64_t*)(ws + w.ranges);
    const DpAny src{dp, dp_fp64};
    prof_begin("k_nufft_fused", st);
    switch (p.kp.w) {
#define MM_FUSED_W(n) case n: fused_w<n>(p, w, ws, S, t, src, t0, scale, ranges, (float2*)coef, ldc, st); break;
        MM_FUSED_W(4) MM_FUSED_W(5) MM_FUSED_W(6) MM_FUSED_W(7) MM_FUSED_W(8) MM_FUSED_W(9) MM_FUSED_W(10)
        MM_FUSED_W(11) MM_FUSED_W(12)
#undef MM_FUSED_W
        default: return hipErrorInvalidValue;
    }
    prof_end("k_nufft_fused", st);
    return hipGetLastError();
}

}  // namespace mm
