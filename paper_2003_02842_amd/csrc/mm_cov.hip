// gfx950 kernels of the Dirichlet / Fejer contraction (Eqs. Der:2, Der:3; steps
// C.1/C.2 of the MM algorithm) and the correlation step.
//
// With real returns c_{-k} = conj(c_k) (Sec. 2.2.2), so
//   Sigma_ij = (2pi)^2 sum_{k=0..N} m_k w_k Re(c_k^i conj c_k^j),  m_0 = 1, m_k = 2,
// a real symmetric product of the D x 2(N+1) matrix X_i,2k+e = s_k (Re,Im)_e c_k^i,
// s_k = 2pi sqrt(m_k w_k), with itself.
//
//   k_cov_small     small D, any number of cutoffs: one workgroup per group of
//                   series, a power of two of lanes per (i, j) pair, FP64 running sums
//                   S0(N) = sum m_k P_k and S1(N) = sum m_k k P_k over k, read off
//                   at every cutoff (Dirichlet S0/(2N+1), Fejer (S0 - S1/N)/(N+1)),
//                   and the correlations of each cutoff in the same launch
//   k_split_bf16    X in BF16 hi/lo parts: hi = rne(x), lo = rne(x - hi)
//   k_syrk_mfma256  lower-triangle 256x256 tiles of X X^T on v_mfma_f32_32x32x16_bf16,
//                   hi*hi + hi*lo + lo*hi with FP32 accumulation, split over k; operand
//                   tiles go HBM -> LDS by global_load_lds, double-buffered
//   k_syrk_mfma     the same on 128x128 tiles (smaller D)
//   k_syrk_reduce   sum of the k-splits, mirrored to the full matrix
//   k_cov_fp64      FP64 tiled product for the plain form
//   k_corr          R_ij = Sigma_ij / sqrt(Sigma_ii Sigma_jj), NaN if a variance <= 0
#include <hip/hip_runtime.h>

#include "mm_bf16.h"
#include "mm_internal.h"

#include <algorithm>
#include <vector>

namespace mm {

static const double kTwoPi = 6.283185307179586476925286766559;

__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }

#ifndef MM_SYRK_XCD_ORDER
#define MM_SYRK_XCD_ORDER 1
#endif

// (split, tile) of a contraction workgroup.  Workgroups are dealt to the eight
// XCDs in turn (workgroup b runs on XCD b mod 8), each XCD with its own L2.  The
// XCD-aware order numbers each XCD's workgroups as one contiguous run of the
// split-major (split, tile) sequence, so the workgroups running side by side on
// an XCD share a k-range and read the same few row blocks of X through its L2,
// instead of every workgroup streaming its own operands from HBM.
__device__ __forceinline__ void syrk_work_item(int b, int ntiles, int nsplit, int& split, int& t)
{
    int q = b;
    if (MM_SYRK_XCD_ORDER) {
        const int nwg = ntiles * nsplit;
        const int per = nwg >> 3, rem = nwg & 7;   // XCD x runs per + (x < rem) workgroups
        const int x = b & 7, r = b >> 3;
        q = x * per + min(x, rem) + r;
    }
    split = q / ntiles;
    t = q - split * ntiles;
}

struct SortedCutoffs {
    int n;
    int N[kMaxCutoffs];      // ascending
    int slot[kMaxCutoffs];   // output slot of each
};

// Small D (D(D+1)/2 pairs per group): one workgroup per group, KL consecutive
// lanes per pair (KL a power of two), each lane taking every KL-th k of a 64-wide
// chunk staged in LDS.  The k range is cut into segments at the cutoffs; at the end
// of a segment the KL lanes of a pair add their partial sums by butterfly shuffles
// into the running S0 = sum m_k P_k and S1 = sum m_k k P_k (m_0 = 1, m_k = 2,
// P_k = Re c_k^(i) conj c_k^(j)), so every cutoff N reads
//   Dirichlet (2pi)^2 S0/(2N+1),  Fejer (2pi)^2 (S0 - S1/N)/(N+1).
// With corr, the correlation of every cutoff (as k_corr computes it, from the
// stored covariances) is written too, after the last k, from copies of every
// cutoff's covariances kept in LDS; the KL lanes of a pair share the cutoffs.
template <typename CT, typename OT>
__global__ void k_cov_small(int D, const CT* __restrict__ coef, int64_t ldc, int Nmax, SortedCutoffs cut, int basis,
                            int G, int kl_bits, OT* __restrict__ cov, OT* __restrict__ corr)
{
    constexpr int KC = 64;
    extern __shared__ __align__(16) char smem_raw[];
    double2* sh = reinterpret_cast<double2*>(smem_raw);   // D x KC
    OT* dg = reinterpret_cast<OT*>(sh + D * KC);           // n x D: the diagonal at each cutoff (with corr)
    OT* vals = dg + cut.n * D;                             // n x npairs: every pair at each cutoff
    const int g = blockIdx.x;
    const int KL = 1 << kl_bits;
    const int npairs = D * (D + 1) / 2;
    const int pidx = (int)threadIdx.x >> kl_bits, lane = (int)threadIdx.x & (KL - 1);
    const bool valid = pidx < npairs;
    int pi = 0, pj = 0;
    if (valid) {
        int i = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
        while (i * (i + 1) / 2 > pidx) --i;
        while ((i + 1) * (i + 2) / 2 <= pidx) ++i;
        pi = i;
        pj = pidx - i * (i + 1) / 2;
    }
    double S0 = 0.0, S1 = 0.0, a0 = 0.0, a1 = 0.0;
    int q = 0;
    const double fourpi2 = kTwoPi * kTwoPi;
    // the next chunk is loaded into registers (at most PF values per thread) while the
    // current one is summed, so its loads are in flight during the arithmetic
    constexpr int PF = 5;
    CT nxt[PF];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int idx = (int)threadIdx.x + u * (int)blockDim.x;
            const int d = idx / KC, kk = idx - d * KC;
            if (idx < D * KC && k0 + kk <= Nmax) nxt[u] = coef[(int64_t)(g * D + d) * ldc + k0 + kk];
            else nxt[u] = CT{0, 0};
        }
    };
    fetch(0);
    for (int k0 = 0; k0 <= Nmax; k0 += KC) {
        const int kc = min(KC, Nmax + 1 - k0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int idx = (int)threadIdx.x + u * (int)blockDim.x;
            if (idx < D * KC) sh[idx] = to_d2(nxt[u]);
        }
        if (k0 + KC <= Nmax) fetch(k0 + KC);
        __syncthreads();
        int kk = 0;
        while (kk < kc) {
            // segment [kk, kend): up to and including the next cutoff, or the chunk's end
            const bool at_cut = q < cut.n && cut.N[q] < k0 + kc;
            const int kend = at_cut ? cut.N[q] - k0 + 1 : kc;
            if (valid) {
                for (int x = kk + lane; x < kend; x += KL) {
                    const double2 u = sh[pi * KC + x], v = sh[pj * KC + x];
                    const double P = u.x * v.x + u.y * v.y;
                    const int k = k0 + x;
                    const double mP = (k ? 2.0 : 1.0) * P;
                    a0 += mP;
                    a1 += (double)k * mP;
                }
            }
            kk = kend;
            if (at_cut) {
                for (int off = KL >> 1; off > 0; off >>= 1) {
                    a0 += __shfl_xor(a0, off);
                    a1 += __shfl_xor(a1, off);
                }
                S0 += a0;
                S1 += a1;
                a0 = a1 = 0.0;
                const int kcut = k0 + kend - 1;
                while (q < cut.n && cut.N[q] == kcut) {
                    if (valid && lane == 0) {
                        const double Nd = (double)kcut;
                        double v = (basis == MM_DIRICHLET) ? S0 / (2.0 * Nd + 1.0) : (S0 - S1 / Nd) / (Nd + 1.0);
                        v *= fourpi2;
                        OT* C = cov + ((int64_t)cut.slot[q] * G + g) * D * D;
                        C[pi * D + pj] = (OT)v;
                        C[pj * D + pi] = (OT)v;
                        if (corr) {
                            vals[q * npairs + pidx] = (OT)v;
                            if (pi == pj) dg[q * D + pi] = (OT)v;
                        }
                    }
                    ++q;
                }
            }
        }
    }
    if (!corr) return;
    __syncthreads();
    if (!valid) return;
    for (q = lane; q < cut.n; q += KL) {
        const int64_t mo = ((int64_t)cut.slot[q] * G + g) * D * D;
        const OT c = vals[q * npairs + pidx], a = dg[q * D + pi], b = dg[q * D + pj];
        const OT r = (a > (OT)0 && b > (OT)0) ? c / (sqrt(a) * sqrt(b)) : (OT)NAN;
        corr[mo + pi * D + pj] = r;
        corr[mo + pj * D + pi] = r;
    }
}

template <typename OT>
__global__ void k_corr(int64_t total, int D, const OT* __restrict__ cov, OT* __restrict__ corr)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    // 64-bit flat indices: D * D exceeds 2^31 once D > 46340
    const int64_t DD = (int64_t)D * D;
    const int64_t m = idx / DD;
    const int64_t r = idx - m * DD;
    const int64_t i = r / D, j = r - i * D;
    const OT* C = cov + m * DD;
    const OT a = C[i * D + i], b = C[j * D + j];
    corr[idx] = (a > (OT)0 && b > (OT)0) ? C[r] / (sqrt(a) * sqrt(b)) : (OT)NAN;
}

// ----------------------------------------------------------------------------------- FP64 plain
constexpr int F64T = 64;   // tile edge
constexpr int F64K = 16;   // k per stage

__global__ __launch_bounds__(256) void k_cov_fp64(int D, const double2* __restrict__ coef, int64_t ldc, int N,
                                                  int basis, double* __restrict__ cov)
{
    __shared__ double2 sA[F64K][F64T + 1];
    __shared__ double2 sB[F64K][F64T + 1];
    // lower-triangle tile enumeration t = bi(bi+1)/2 + bj
    const int t = blockIdx.x;
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    double acc[4][4];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    const double fourpi2 = kTwoPi * kTwoPi;
    for (int k0 = 0; k0 <= N; k0 += F64K) {
        for (int idx = threadIdx.x; idx < F64T * F64K; idx += 256) {
            int r = idx >> 4, kk = idx & 15;
            int k = k0 + kk;
            double wk = 0.0;
            if (k <= N) {
                double w = (basis == MM_DIRICHLET) ? 1.0 / (2.0 * N + 1.0)
                                                   : (1.0 - (double)k / (double)N) / ((double)N + 1.0);
                wk = (k ? 2.0 : 1.0) * w * fourpi2;
            }
            int ia = bi * F64T + r, ib = bj * F64T + r;
            double2 a = (k <= N && ia < D) ? coef[(int64_t)ia * ldc + k] : make_double2(0.0, 0.0);
            double2 b = (k <= N && ib < D) ? coef[(int64_t)ib * ldc + k] : make_double2(0.0, 0.0);
            sA[kk][r] = make_double2(a.x * wk, a.y * wk);
            sB[kk][r] = b;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < F64K; ++kk) {
            double2 a[4], b[4];
            for (int u = 0; u < 4; ++u) a[u] = sA[kk][ty * 4 + u];
            for (int v = 0; v < 4; ++v) b[v] = sB[kk][tx * 4 + v];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u].x, b[v].x, fma(a[u].y, b[v].y, acc[u][v]));
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            int i = bi * F64T + ty * 4 + u, j = bj * F64T + tx * 4 + v;
            // i >= j only: (i, j) and (j, i) take one value, so Sigma is exactly symmetric
            if (i < D && j <= i) {
                cov[(int64_t)i * D + j] = acc[u][v];
                cov[(int64_t)j * D + i] = acc[u][v];
            }
        }
}

// ------------------------------------------------------------------------------ split-BF16 MFMA
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int ST = 128;         // output tile edge
constexpr int SK = 32;          // k (real columns) per LDS stage
constexpr int SLD = SK + 8;     // padded LDS row, bf16 elements


// X (Dp x Kp, zero padded) from float2 coefficients: column 2k+e = s_k (Re, Im)_e c_k.
// Column scale of X: s_k = 2pi sqrt(m_k w_k) for k <= N (FP64, rounded once), 0 on
// the padding, so that the split reads one float per column instead of forming
// the weight per element.
__global__ void k_split_scale(int N, int basis, int64_t Kh, float* __restrict__ scale)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Kh) return;
    float v = 0.f;
    if (k <= N) {
        const double Nd = (double)N;
        const double w = (basis == MM_DIRICHLET) ? 1.0 / (2.0 * Nd + 1.0) : (1.0 - (double)k / Nd) / (Nd + 1.0);
        v = (float)(kTwoPi * sqrt((k ? 2.0 : 1.0) * w));
    }
    scale[k] = v;
}

__global__ void k_split_bf16(int D, const float2* __restrict__ coef, int64_t ldc, int N,
                             const float* __restrict__ scale, int64_t Kp, uint16_t* __restrict__ hi,
                             uint16_t* __restrict__ lo)
{
    const int64_t row = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < Kp / 2; c += (int64_t)gridDim.x * blockDim.x) {
        float2 cc = make_float2(0.f, 0.f);
        float sc = 0.f;
        const int k = (int)c;
        if (row < D && k <= N) {
            sc = scale[k];
            cc = coef[row * ldc + k];
        }
        uint32_t h, l;
        bf16_split_pair(cc.x, cc.y, sc, h, l);
        *(uint32_t*)&hi[row * Kp + 2 * c] = h;
        *(uint32_t*)&lo[row * Kp + 2 * c] = l;
    }
}

// One workgroup = one lower-triangle 128x128 tile over one k-range, numbered in
// the XCD-aware order of syrk_work_item, so that the tiles sharing a row panel
// read it through one XCD's L2.
__global__ __launch_bounds__(256) void k_syrk_mfma(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo,
                                                   const uint16_t* __restrict__ bhi, const uint16_t* __restrict__ blo,
                                                   int64_t Kp, int64_t kchunk, int ntiles, int nsplit,
                                                   float* __restrict__ partial, const int32_t* __restrict__ kstep)
{
    __shared__ __align__(16) uint16_t sAh[ST * SLD];
    __shared__ __align__(16) uint16_t sAl[ST * SLD];
    __shared__ __align__(16) uint16_t sBh[ST * SLD];
    __shared__ __align__(16) uint16_t sBl[ST * SLD];
    int split, t;
    syrk_work_item((int)blockIdx.x, ntiles, nsplit, split, t);
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    // k-range of this split: equal chunks, or (kstep given) k-steps kstep[2 split] .. kstep[2 split + 1]
    const int64_t kb = kstep ? (int64_t)kstep[2 * split] * SK : (int64_t)split * kchunk;
    const int64_t ke = kstep ? (int64_t)kstep[2 * split + 1] * SK : min(kb + kchunk, Kp);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const uint16_t* Ah = hi + (int64_t)bi * ST * Kp;
    const uint16_t* Al = lo + (int64_t)bi * ST * Kp;
    const uint16_t* Bh = bhi + (int64_t)bj * ST * Kp;
    const uint16_t* Bl = blo + (int64_t)bj * ST * Kp;
    f32x16 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
    // each thread moves rows tid>>2 and 64 + (tid>>2), 16-byte chunk tid&3, of all four arrays
    const int row0 = tid >> 2, ch = tid & 3;
    for (int64_t k0 = kb; k0 < ke; k0 += SK) {
        // 128 rows x 32 bf16 = 512 chunks of 16 B per array
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = row0 + 64 * h;
            const int64_t go = (int64_t)row * Kp + k0 + ch * 8;
            const int l_ = row * SLD + ch * 8;
            *(uint4*)&sAh[l_] = *(const uint4*)&Ah[go];
            *(uint4*)&sAl[l_] = *(const uint4*)&Al[go];
            *(uint4*)&sBh[l_] = *(const uint4*)&Bh[go];
            *(uint4*)&sBl[l_] = *(const uint4*)&Bl[go];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < SK; ks += 16) {
            bf16x8 fah[2], fal[2], fbh[2], fbl[2];
            const int kof = ks + 8 * (lane >> 5);
            for (int a = 0; a < 2; ++a) {
                const int r = wy * 64 + a * 32 + (lane & 31);
                fah[a] = *(const bf16x8*)&sAh[r * SLD + kof];
                fal[a] = *(const bf16x8*)&sAl[r * SLD + kof];
            }
            for (int b = 0; b < 2; ++b) {
                const int c = wx * 64 + b * 32 + (lane & 31);
                fbh[b] = *(const bf16x8*)&sBh[c * SLD + kof];
                fbl[b] = *(const bf16x8*)&sBl[c * SLD + kof];
            }
            // the three products of one block are four MFMAs apart
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[a], fbh[b], acc[a][b], 0, 0, 0);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[a], fbl[b], acc[a][b], 0, 0, 0);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[a], fbh[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    float* P = partial + ((int64_t)split * ntiles + t) * ST * ST;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int r = 0; r < 16; ++r) {
                const int i = wy * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = wx * 64 + b * 32 + (lane & 31);
                P[i * ST + j] = acc[a][b][r];
            }
}

// Large-D form: one workgroup = one lower-triangle 256x256 tile over one k-range;
// each of the four waves owns a 128x128 quadrant (4 x 4 blocks of 32 x 32, 256
// accumulators per lane).  Stages of 32 k move global -> registers -> LDS with
// two LDS buffers, so the loads of stage s+1 are in flight while stage s runs on
// MFMA.  LDS rows are 64 bytes (4 chunks of 16 B); chunk c of row r sits at
// position c ^ ((r >> 2) & 3), which keeps every 16-lane group of a 16-byte
// fragment read on distinct banks.  A diagonal tile stages its one panel once
// and leaves the quadrant above the diagonal idle.
constexpr int T2 = 256;
constexpr int SK2 = 32;

__device__ __forceinline__ int swz(int row, int chunk) { return (row << 2) | (chunk ^ ((row >> 2) & 3)); }

// Stage loads: one global_load_lds_dwordx4 per wave fills 1 KB (16 rows of an
// array); lane p lands in slot p, i.e. row R0 + (p >> 2), physical chunk p & 3, so
// it fetches logical chunk (p & 3) ^ ((row >> 2) & 3).  Byte offsets fit 32 bits.
__device__ __forceinline__ void syrk256_load(uint4* L, const char* const (&src)[4], const uint32_t (&goff)[4],
                                             uint32_t kbyte, int wave, bool diag)
{
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (a >= 2 && diag) break;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            __builtin_amdgcn_global_load_lds(src[a] + goff[q] + kbyte, L + (a * T2 + 16 * (4 * wave + q)) * 4, 16,
                                             0, 0);
    }
}

#ifndef MM_SYRK_INTERLEAVE
#define MM_SYRK_INTERLEAVE 1
#endif
#ifndef MM_SYRK_LPG
#define MM_SYRK_LPG 4
#endif

// One stage (32 k) of a wave's 128x128 quadrant from LDS buffer L: per 16 k, the
// four A row blocks (hi, lo) stay in registers while each B block streams through.
// If `load`, the next stage's operands stream into Ln meanwhile, MM_SYRK_LPG loads
// before each of the first blocks rather than all at once: a burst fills the
// memory queue and holds the wave at issue until most of it has landed, so the
// products would wait for the transfer.  The scheduling barriers keep the compiler
// from gathering the loads again.  A diagonal tile loads only its A panel (arrays
// 0 and 1).
__device__ __forceinline__ void syrk256_stage_dma(const uint4* __restrict__ L, uint4* Ln, bool load, bool diag,
                                                  const char* const (&src)[4], const uint32_t (&goff)[4],
                                                  uint32_t kbyte, int ba, int wy, int wx, int lane, int wave,
                                                  f32x16 (&acc)[4][4])
{
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int ch = 2 * ks + (lane >> 5);
        bf16x8 fah[4], fal[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int r = wy * 128 + a * 32 + (lane & 31);
            uint4 vh = L[0 * T2 * 4 + swz(r, ch)], vl = L[1 * T2 * 4 + swz(r, ch)];
            fah[a] = *reinterpret_cast<bf16x8*>(&vh);
            fal[a] = *reinterpret_cast<bf16x8*>(&vl);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = wx * 128 + b * 32 + (lane & 31);
            uint4 vh = L[ba * T2 * 4 + swz(r, ch)], vl = L[(ba + 1) * T2 * 4 + swz(r, ch)];
            if (MM_SYRK_INTERLEAVE) {
                // 16 loads (array arr, row group q) in groups of LPG before the blocks
                constexpr int LPG = MM_SYRK_LPG;
                const int g = ks * 4 + b;
                if (load && g * LPG < 16) {
#pragma unroll
                    for (int u = 0; u < LPG; ++u) {
                        const int li = g * LPG + u, arr = li >> 2, q = li & 3;
                        if (arr < 2 || !diag)
                            __builtin_amdgcn_global_load_lds(src[arr] + goff[q] + kbyte,
                                                             Ln + (arr * T2 + 16 * (4 * wave + q)) * 4, 16, 0, 0);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            const bf16x8 fbh = *reinterpret_cast<bf16x8*>(&vh), fbl = *reinterpret_cast<bf16x8*>(&vl);
            // the three products of one block are four MFMAs apart, so no MFMA waits on
            // the accumulator of the one before it
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[a], fbh, acc[a][b], 0, 0, 0);
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fah[a], fbl, acc[a][b], 0, 0, 0);
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fal[a], fbh, acc[a][b], 0, 0, 0);
        }
    }
}

__global__ __launch_bounds__(256) void k_syrk_mfma256(const uint16_t* __restrict__ hi,
                                                      const uint16_t* __restrict__ lo,
                                                      const uint16_t* __restrict__ bhi,
                                                      const uint16_t* __restrict__ blo, int64_t Kp, int64_t kchunk,
                                                      int ntiles, int nsplit, float* __restrict__ partial,
                                                      const int32_t* __restrict__ kstep)
{
    __shared__ uint4 lds0[4 * T2 * 4];   // [array: A hi, A lo, B hi, B lo][row][chunk], even stages
    __shared__ uint4 lds1[4 * T2 * 4];   // odd stages
    int split, t;
    syrk_work_item((int)blockIdx.x, ntiles, nsplit, split, t);
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    // a diagonal tile of X X^T (B the same arrays as A) stages one panel and skips
    // its upper quadrant; a product A B^T with B of its own computes every quadrant
    const bool diag = bi == bj && bhi == hi;
    // k-range of this split: equal chunks, or (kstep given) k-steps kstep[2 split] .. kstep[2 split + 1]
    const int64_t kb = kstep ? (int64_t)kstep[2 * split] * SK2 : (int64_t)split * kchunk;
    const int64_t ke = kstep ? (int64_t)kstep[2 * split + 1] * SK2 : min(kb + kchunk, Kp);
    const int nst = (int)((ke - kb) / SK2);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wy = wave >> 1, wx = wave & 1;
    const bool active = !(diag && wy == 0 && wx == 1);
    const char* const src[4] = {(const char*)(hi + (int64_t)bi * T2 * Kp), (const char*)(lo + (int64_t)bi * T2 * Kp),
                                (const char*)(bhi + (int64_t)bj * T2 * Kp), (const char*)(blo + (int64_t)bj * T2 * Kp)};
    uint32_t goff[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = 16 * (4 * wave + q) + (lane >> 2);
        goff[q] = (uint32_t)(row * Kp + 8 * ((lane & 3) ^ ((row >> 2) & 3))) * 2u;
    }
    f32x16 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;
    const int ba = diag ? 0 : 2;   // arrays holding the B panel
    const uint32_t kb0 = (uint32_t)kb * 2u;
    // The wave holding the upper quadrant of a diagonal tile only loads.  Stage s reads buffer s mod 2 while stage s+1 loads into the other; the two
    // buffers are addressed statically (a pair of stages per iteration) so that the
    // compiler sees that the loads never touch the buffer being read.
    if (nst > 0) syrk256_load(lds0, src, goff, kb0, wave, diag);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int s = 0; s < nst; s += 2) {
        const bool l1 = s + 1 < nst;
        if (!MM_SYRK_INTERLEAVE && l1) syrk256_load(lds1, src, goff, kb0 + (uint32_t)(s + 1) * SK2 * 2u, wave, diag);
        if (active)
            syrk256_stage_dma(lds0, lds1, l1, diag, src, goff, kb0 + (uint32_t)(s + 1) * SK2 * 2u, ba, wy, wx, lane,
                              wave, acc);
        else if (MM_SYRK_INTERLEAVE && l1)
            syrk256_load(lds1, src, goff, kb0 + (uint32_t)(s + 1) * SK2 * 2u, wave, diag);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (!l1) break;
        const bool l2 = s + 2 < nst;
        if (!MM_SYRK_INTERLEAVE && l2) syrk256_load(lds0, src, goff, kb0 + (uint32_t)(s + 2) * SK2 * 2u, wave, diag);
        if (active)
            syrk256_stage_dma(lds1, lds0, l2, diag, src, goff, kb0 + (uint32_t)(s + 2) * SK2 * 2u, ba, wy, wx, lane,
                              wave, acc);
        else if (MM_SYRK_INTERLEAVE && l2)
            syrk256_load(lds0, src, goff, kb0 + (uint32_t)(s + 2) * SK2 * 2u, wave, diag);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
    if (!active) return;
    float* P = partial + ((int64_t)split * ntiles + t) * T2 * T2;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = wy * 128 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = wx * 128 + b * 32 + (lane & 31);
                P[i * T2 + j] = acc[a][b][r];
            }
}

// Sum of the k-range partials of 16 rows x 64 columns of a lower-triangle tile
// (workgroup = tile, 64x64 sub-block, quarter of it), written to Sigma at (i, j)
// and, through an LDS transpose, at (j, i).  Each thread keeps four partial sums
// so that four loads of the split are in flight at once.
template <int TS>
__global__ __launch_bounds__(256) void k_syrk_reduce(const float* __restrict__ partial, int nsplit, int ntiles, int D,
                                                     float* __restrict__ cov, const int32_t* __restrict__ perm)
{
    // row i of the product is series perm[i] (the identity when perm is NULL)
    auto at = [&](int i, int j) -> int64_t {
        return perm ? (int64_t)perm[i] * D + perm[j] : (int64_t)i * D + j;
    };
    constexpr int ST = TS;
    constexpr int QN = TS / 64;   // 64 x 64 sub-blocks per tile edge
    constexpr int RB = 16;        // rows per workgroup
    __shared__ float tileT[RB][65];
    const int per_tile = QN * QN * (64 / RB);
    const int t = blockIdx.x / per_tile, rem = blockIdx.x % per_tile;
    const int quad = rem / (64 / RB), part = rem % (64 / RB);
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int qi = (quad / QN) * 64, qj = (quad % QN) * 64;
    if (bi == bj && qi < qj) return;   // above the diagonal of a diagonal tile: mirrored from below
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t tstride = (int64_t)ntiles * ST * ST;
    const float* P = partial + (int64_t)t * ST * ST;
    for (int r = ty; r < RB; r += 4) {
        const int li = qi + part * RB + r, lj = qj + tx;
        const float* p = P + li * ST + lj;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        int q = 0;
        for (; q + 3 < nsplit; q += 4) {
            a0 += p[q * tstride];
            a1 += p[(q + 1) * tstride];
            a2 += p[(q + 2) * tstride];
            a3 += p[(q + 3) * tstride];
        }
        for (; q < nsplit; ++q) a0 += p[q * tstride];
        const float acc = (a0 + a1) + (a2 + a3);
        const int i = bi * ST + li, j = bj * ST + lj;
        if (bi == bj) {
            // diagonal tile: (i, j) and (j, i) both come from the lower entry, so that
            // Sigma is exactly symmetric (the MFMA sums the two in different orders)
            if (i < D && j <= i) {
                cov[at(i, j)] = acc;
                cov[at(j, i)] = acc;
            }
            continue;
        }
        if (i < D && j < D) cov[at(i, j)] = acc;
        tileT[r][tx] = acc;
    }
    if (bi == bj) return;
    __syncthreads();
    // rows j = bj*ST + qj + c (c < 64) of Sigma, columns i = bi*ST + qi + part*RB + r (r < RB)
    for (int e = threadIdx.x; e < 64 * RB; e += 256) {
        const int c = e / RB, r = e % RB;
        const int j = bj * ST + qj + c, i = bi * ST + qi + part * RB + r;
        if (i < D && j < D) cov[at(j, i)] = tileT[r][c];
    }
}

// Pairwise cutoffs: entry (i, j) of group g from the sweep slice of cutoff
// N_ij = min(N_i, N_j), and R_ij from the same slice's variances.
template <typename OT>
__global__ void k_pairwise_select(int64_t total, int D, int G, const int32_t* __restrict__ qidx,
                                  const OT* __restrict__ sweep, OT* __restrict__ cov, OT* __restrict__ corr)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t DD = (int64_t)D * D;   // 64-bit flat indices, as in k_corr
    const int64_t g = idx / DD;
    const int64_t r = idx - g * DD;
    const int64_t i = r / D, j = r - i * D;
    const int qi = qidx[i], qj = qidx[j];
    const int q = qi < qj ? qi : qj;     // slices ascend with the cutoff
    const OT* Sq = sweep + ((int64_t)q * G + g) * DD;
    const OT v = Sq[r];
    cov[idx] = v;
    if (corr) {
        const OT a = Sq[i * D + i], b = Sq[j * D + j];
        corr[idx] = (a > (OT)0 && b > (OT)0) ? v / (sqrt(a) * sqrt(b)) : (OT)NAN;
    }
}

hipError_t launch_pairwise_select(int prec, int32_t G, int32_t D, const int32_t* qidx, const void* sweep, void* cov,
                                  void* corr, hipStream_t st)
{
    const int64_t total = (int64_t)G * D * D;
    const int blocks = (int)((total + 255) / 256);
    if (prec == MM_MIXED)
        hipLaunchKernelGGL(k_pairwise_select<float>, dim3(blocks), dim3(256), 0, st, total, D, G, qidx,
                           (const float*)sweep, (float*)cov, (float*)corr);
    else
        hipLaunchKernelGGL(k_pairwise_select<double>, dim3(blocks), dim3(256), 0, st, total, D, G, qidx,
                           (const double*)sweep, (double*)cov, (double*)corr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ per-pair cutoffs
// With per-asset cutoffs (Sec. 3), pair (i, j) is estimated at N_ij = min(N_i, N_j).
// Rows are taken in ascending order of cutoff (row r is series perm[r], cutoff
// Nr[r]), so that for r >= q the pair's cutoff is the column's, N_q, and
//   Sigma_rq = (2pi)^2 sum_{k <= N_q} m_k w_k(N_q) Re(c^r_k conj c^q_k) = sum_k A_rk B_qk
// with A_rk = 2pi sqrt(m_k) c^r_k (k <= N_r) and B_qk = 2pi sqrt(m_k) w_k(N_q) c^q_k
// (k <= N_q): one product A B^T over the lower triangle, however many distinct
// cutoffs there are.  The weights: Dirichlet 1/(2N+1), Fejer (1 - k/N)/(N+1).

// A and B of one group as BF16 hi/lo pairs (row = sorted position, column pair k).
__global__ void k_pair_split(int D, const float2* __restrict__ coef, int64_t ldc, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ Nr, int basis, int64_t Kp, uint32_t* __restrict__ ahi,
                             uint32_t* __restrict__ alo, uint32_t* __restrict__ bhi, uint32_t* __restrict__ blo)
{
    const int row = blockIdx.y;                        // < Dp
    const bool real_row = row < D;
    const int src = real_row ? perm[row] : 0;
    const int N = real_row ? Nr[row] : -1;
    // per-row weight constants in FP64: w_k = w0 (Dirichlet) or (1 - k/N) w0 (Fejer)
    const double w0 = basis == MM_DIRICHLET ? 1.0 / (2.0 * N + 1.0) : 1.0 / (N + 1.0);
    const double invN = 1.0 / (double)N;
    const float two_pi = (float)kTwoPi, two_pi_r2 = (float)(kTwoPi * 1.4142135623730950488);
    const int64_t kp2 = Kp / 2;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < kp2; c += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)c;
        float2 cc = make_float2(0.f, 0.f);
        float sa = 0.f, sb = 0.f;
        if (real_row && k <= N) {
            cc = coef[(int64_t)src * ldc + k];
            sa = k ? two_pi_r2 : two_pi;                  // 2pi sqrt(m_k)
            const double w = basis == MM_DIRICHLET ? w0 : (1.0 - (double)k * invN) * w0;
            sb = (float)((k ? kTwoPi * 1.4142135623730950488 : kTwoPi) * w);
        }
        uint32_t h, l;
        const int64_t at = (int64_t)row * kp2 + c;
        bf16_split_pair(cc.x, cc.y, sa, h, l);
        ahi[at] = h;
        alo[at] = l;
        bf16_split_pair(cc.x, cc.y, sb, h, l);
        bhi[at] = h;
        blo[at] = l;
    }
}

// Variances at every distinct cutoff up to a row's own: one wave per (group, row)
// scans k = 0..N_r with FP64 running sums S0 = sum m_k |c_k|^2 and
// S1 = sum m_k k |c_k|^2 (an inclusive scan over each 64 k, plus the carry); the
// lane at k = N_q (cutq[k] = q) writes var[row][q], Dirichlet (2pi)^2 S0/(2N+1) or
// Fejer (2pi)^2 (S0 - S1/N)/(N+1).
template <typename CT, typename OT>
__global__ __launch_bounds__(64) void k_pair_var(int D, const CT* __restrict__ coef, int64_t ldc,
                                                 const int32_t* __restrict__ perm, const int32_t* __restrict__ Nr,
                                                 const int32_t* __restrict__ cutq, int nq, int basis,
                                                 OT* __restrict__ var)
{
    const int row = blockIdx.x, g = blockIdx.y;
    const int lane = (int)threadIdx.x;
    const int N = Nr[row];
    const CT* c = coef + ((int64_t)g * D + perm[row]) * ldc;
    OT* out = var + ((int64_t)g * D + row) * nq;
    const double fourpi2 = kTwoPi * kTwoPi;
    double carry0 = 0.0, carry1 = 0.0;
    for (int k0 = 0; k0 <= N; k0 += 64) {
        const int k = k0 + lane;
        double v0 = 0.0;
        if (k <= N) {
            const double2 u = to_d2(c[k]);
            v0 = (k ? 2.0 : 1.0) * (u.x * u.x + u.y * u.y);
        }
        double v1 = (double)k * v0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double a0 = __shfl_up(v0, o), a1 = __shfl_up(v1, o);
            if (lane >= o) {
                v0 += a0;
                v1 += a1;
            }
        }
        const double S0 = carry0 + v0, S1 = carry1 + v1;
        if (k <= N) {
            const int q = cutq[k];
            if (q >= 0) {
                const double Nd = (double)k;
                const double v = basis == MM_DIRICHLET ? S0 / (2.0 * Nd + 1.0) : (S0 - S1 / Nd) / (Nd + 1.0);
                out[q] = (OT)(fourpi2 * v);
            }
        }
        carry0 = __shfl(S0, 63);
        carry1 = __shfl(S1, 63);
    }
}

// Correlations of the pairwise estimates: entry (a, b) at N_ab from the variances
// of both series at that cutoff (the slot of the lower-ranked series' cutoff);
// on the diagonal Sigma_aa / (sqrt Sigma_aa)^2.  NaN for a non-positive variance.
template <typename OT>
__global__ void k_pair_corr(int64_t total, int D, const int32_t* __restrict__ rank, const int32_t* __restrict__ slot,
                            const OT* __restrict__ var, int nq, const OT* __restrict__ cov, OT* __restrict__ corr)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t DD = (int64_t)D * D;
    const int64_t g = idx / DD;
    const int64_t r = idx - g * DD;
    const int a = (int)(r / D), b = (int)(r - (int64_t)a * D);
    const OT v = cov[idx];
    OT va, vb;
    if (a == b) {
        va = vb = v;
    } else {
        const int ra = rank[a], rb = rank[b];
        const int q = slot[min(ra, rb)];
        va = var[((int64_t)g * D + ra) * nq + q];
        vb = var[((int64_t)g * D + rb) * nq + q];
    }
    corr[idx] = (va > (OT)0 && vb > (OT)0) ? v / (sqrt(va) * sqrt(vb)) : (OT)NAN;
}

// The FP64 form of the per-pair product: lower-triangle 64 x 64 tiles over the
// sorted rows, A unweighted, B = (2pi)^2 m_k w_k(N_q) c^q_k, written to the
// series' own positions (both halves).
__global__ __launch_bounds__(256) void k_pair_fp64(int D, const double2* __restrict__ coef, int64_t ldc, int Nmax,
                                                   const int32_t* __restrict__ perm, const int32_t* __restrict__ Nr,
                                                   int basis, double* __restrict__ cov)
{
    __shared__ double2 sA[F64K][F64T + 1];
    __shared__ double2 sB[F64K][F64T + 1];
    const int t = blockIdx.x;
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    double acc[4][4];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    const double fourpi2 = kTwoPi * kTwoPi;
    for (int k0 = 0; k0 <= Nmax; k0 += F64K) {
        for (int idx = threadIdx.x; idx < F64T * F64K; idx += 256) {
            const int r = idx >> 4, kk = idx & 15;
            const int k = k0 + kk;
            const int ia = bi * F64T + r, ib = bj * F64T + r;
            double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
            if (ia < D && k <= Nr[ia]) a = coef[(int64_t)perm[ia] * ldc + k];
            if (ib < D && k <= Nr[ib]) {
                const double N = (double)Nr[ib];
                const double w = basis == MM_DIRICHLET ? 1.0 / (2.0 * N + 1.0) : (1.0 - (double)k / N) / (N + 1.0);
                const double wk = (k ? 2.0 : 1.0) * w * fourpi2;
                const double2 bb = coef[(int64_t)perm[ib] * ldc + k];
                b = make_double2(bb.x * wk, bb.y * wk);
            }
            sA[kk][r] = a;
            sB[kk][r] = b;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < F64K; ++kk) {
            double2 a[4], b[4];
            for (int u = 0; u < 4; ++u) a[u] = sA[kk][ty * 4 + u];
            for (int v = 0; v < 4; ++v) b[v] = sB[kk][tx * 4 + v];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u].x, b[v].x, fma(a[u].y, b[v].y, acc[u][v]));
        }
        __syncthreads();
    }
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            const int i = bi * F64T + ty * 4 + u, j = bj * F64T + tx * 4 + v;
            if (i < D && j <= i) {   // r >= q: the column's cutoff is the pair's
                cov[(int64_t)perm[i] * D + perm[j]] = acc[u][v];
                cov[(int64_t)perm[j] * D + perm[i]] = acc[u][v];
            }
        }
}

// ------------------------------------------------------------------------------- launchers
static SortedCutoffs sort_cutoffs(const Cutoffs& c)
{
    SortedCutoffs s;
    s.n = c.n;
    for (int i = 0; i < c.n; ++i) { s.N[i] = c.N[i]; s.slot[i] = i; }
    for (int i = 1; i < c.n; ++i)
        for (int j = i; j > 0 && s.N[j - 1] > s.N[j]; --j) {
            int a = s.N[j]; s.N[j] = s.N[j - 1]; s.N[j - 1] = a;
            int b = s.slot[j]; s.slot[j] = s.slot[j - 1]; s.slot[j - 1] = b;
        }
    return s;
}

hipError_t launch_cov_small(int prec, int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t Nmax,
                            const Cutoffs& cut, int basis, void* cov, hipStream_t st, void* corr)
{
    SortedCutoffs sc = sort_cutoffs(cut);
    const int npairs = D * (D + 1) / 2;
    // lanes per pair: as many as keep the workgroup within 512 threads (<= 64, one wave)
    int kl_bits = 0;
    while (kl_bits < 6 && npairs * (2 << kl_bits) <= 512) ++kl_bits;
    const int threads = std::max(64, ((npairs << kl_bits) + 63) / 64 * 64);
    if (D * 64 > 5 * threads) return hipErrorInvalidValue;   // k_cov_small stages at most 5 values per thread
    // the correlations in the same launch while every cutoff's values fit in LDS
    const size_t os = prec == MM_MIXED ? sizeof(float) : sizeof(double);
    const size_t lds_corr = (size_t)sc.n * (D + npairs) * os;
    const bool fold = corr && (size_t)D * 64 * sizeof(double2) + lds_corr <= 64 * 1024;
    const size_t lds = (size_t)D * 64 * sizeof(double2) + (fold ? lds_corr : 0);
    void* kc = fold ? corr : nullptr;
    prof_begin("k_cov_small", st);
    if (prec == MM_MIXED)
        hipLaunchKernelGGL((k_cov_small<float2, float>), dim3(G), dim3(threads), lds, st, D, (const float2*)coef, ldc,
                           Nmax, sc, basis, G, kl_bits, (float*)cov, (float*)kc);
    else
        hipLaunchKernelGGL((k_cov_small<double2, double>), dim3(G), dim3(threads), lds, st, D, (const double2*)coef,
                           ldc, Nmax, sc, basis, G, kl_bits, (double*)cov, (double*)kc);
    prof_end("k_cov_small", st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && corr && !fold) e = launch_corr(prec, (int64_t)cut.n * G, D, cov, corr, st);
    return e;
}

hipError_t launch_corr(int prec, int64_t mats, int32_t D, const void* cov, void* corr, hipStream_t st)
{
    const int64_t total = mats * D * D;
    if (total == 0) return hipSuccess;
    const int blocks = (int)((total + 255) / 256);
    prof_begin("k_corr", st);
    if (prec == MM_MIXED)
        hipLaunchKernelGGL(k_corr<float>, dim3(blocks), dim3(256), 0, st, total, D, (const float*)cov, (float*)corr);
    else
        hipLaunchKernelGGL(k_corr<double>, dim3(blocks), dim3(256), 0, st, total, D, (const double*)cov,
                           (double*)corr);
    prof_end("k_corr", st);
    return hipGetLastError();
}

hipError_t launch_cov_fp64(int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t N, int basis, void* cov,
                           hipStream_t st)
{
    const int tn = (D + F64T - 1) / F64T;
    const int ntiles = tn * (tn + 1) / 2;
    for (int g = 0; g < G; ++g) {
        prof_begin("k_cov_fp64", st);
        hipLaunchKernelGGL(k_cov_fp64, dim3(ntiles), dim3(256), 0, st, D,
                           (const double2*)coef + (int64_t)g * D * ldc, ldc, N, basis,
                           (double*)cov + (int64_t)g * D * D);
        prof_end("k_cov_fp64", st);
    }
    return hipGetLastError();
}

#ifndef MM_SYRK_BIG_TILES
#define MM_SYRK_BIG_TILES 1
#endif

struct MfmaShape {
    int ts;               // tile edge: 128 or 256
    int tn, ntiles, nsplit;
    int64_t Dp, Kp, kchunk;
    size_t hi, lo, partial, scale, fac, total;
};

// k-ranges per 256-wide tile: the workgroups (tiles x ranges) run in rounds of 256
// (one per CU), so the time goes as ceil(tiles s / 256) / s of one tile's full k
// range, plus the partial tiles each range writes and the reduce reads back.  The
// smallest s within 10% of the best modelled time wins (shorter ranges cost more
// than the model counts: D = 3000 measured slower at 13 ranges than at 3), and
// each range keeps >= 64 stages.  Model rates: 4.7 TFLOP/s of products per CU,
// 5 TB/s for the partials.
static int split_count(int ntiles, int64_t Kp)
{
    const double c_k = 256.0 * 256.0 * 6.0 / 4.7e12;      // s per k column of one tile on one CU
    const double c_p = 2.0 * 256.0 * 256.0 * 4.0 / 5.0e12;   // s per partial tile written and read
    int best_s = 1;
    double best_t = 0.0;
    for (int sp = 1; sp <= 64; ++sp) {
        if (sp > 1 && Kp / sp < 64 * SK2) break;
        const double rounds = (double)((ntiles * (int64_t)sp + 255) / 256);
        const double t = rounds / sp * (double)Kp * c_k + (double)sp * ntiles * c_p;
        if (sp == 1 || t < 0.90 * best_t) {
            best_s = sp;
            best_t = t;
        }
    }
    return best_s;
}

static MfmaShape mfma_shape(int32_t D, int32_t N, SyrkChoice sc = {})
{
    MfmaShape s;
    s.Kp = ((2ll * (N + 1) + SK - 1) / SK) * SK;
    const int tn2 = (D + T2 - 1) / T2;
    // the 256-wide kernel addresses a panel with 32-bit byte offsets (row x Kp x 2 for
    // rows < 256, plus the k offset); beyond that the 128-wide kernel (64-bit) runs
    const bool offsets32 = (s.Kp * 2) * 257 < (1ll << 32);
    const bool big = sc.tile == 256 ? offsets32
                   : sc.tile == 128 ? false
                                    : (MM_SYRK_BIG_TILES && tn2 >= 4 && s.Kp / SK2 >= 64 && offsets32);
    if (big) {
        // 256-wide tiles, about one workgroup per CU, so every tile's k-range runs
        // concurrently and the partials stay few
        s.ts = T2;
        s.tn = tn2;
        s.ntiles = s.tn * (s.tn + 1) / 2;
        s.Dp = (int64_t)s.tn * T2;
        s.nsplit = sc.splits > 0 ? (int)std::min<int64_t>(sc.splits, s.Kp / SK2) : split_count(s.ntiles, s.Kp);
        const int64_t per = (s.Kp + s.nsplit - 1) / s.nsplit;
        s.kchunk = ((per + SK2 - 1) / SK2) * SK2;
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        size_t o = 0;
        s.hi = o; o += al((size_t)s.Dp * s.Kp * 2);
        s.lo = o; o += al((size_t)s.Dp * s.Kp * 2);
        s.partial = o; o += al((size_t)s.nsplit * s.ntiles * T2 * T2 * 4);
        s.scale = o; o += al((size_t)s.Kp / 2 * 4);
        s.fac = o; o += al((size_t)s.Kp / 2 * 4);
        s.total = o;
        return s;
    }
    s.ts = ST;
    s.tn = (D + ST - 1) / ST;
    s.ntiles = s.tn * (s.tn + 1) / 2;
    s.Dp = (int64_t)s.tn * ST;
    // k-ranges: 8 m of them, m per XCD.  One per XCD measured fastest once the
    // tiles alone give a few hundred workgroups; small D takes more ranges (each
    // >= 8 k-stages) to occupy the chip.
    const int64_t ksteps = s.Kp / SK;
    int best_m = (int)((512 + 8ll * s.ntiles - 1) / (8ll * s.ntiles));
    const int max_m = (int)std::max<int64_t>(1, ksteps / 64);
    best_m = std::max(1, std::min(best_m, max_m));
    // never more ranges than k-stages (an empty range would still write a partial tile)
    s.nsplit = (int)std::min<int64_t>(sc.splits > 0 ? sc.splits : 8 * best_m, ksteps);
    int64_t per = (s.Kp + s.nsplit - 1) / s.nsplit;
    s.kchunk = ((per + SK - 1) / SK) * SK;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    s.hi = o; o += al((size_t)s.Dp * s.Kp * 2);
    s.lo = o; o += al((size_t)s.Dp * s.Kp * 2);
    s.partial = o; o += al((size_t)s.nsplit * s.ntiles * ST * ST * 4);
    s.scale = o; o += al((size_t)s.Kp / 2 * 4);
    s.fac = o; o += al((size_t)s.Kp / 2 * 4);
    s.total = o;
    return s;
}

// ---------------------------------------------------------------- MFMA N sweep
// Every cutoff N_1 < ... < N_n of a sweep from one pass over k (Eqs. Der:2/3).
// The operands hold the k of segment j, (N_{j-1}, N_j], in a column block of its
// own padded to the product's k-step, and the product's k-ranges never cross a
// segment, so every partial tile is a Gram matrix of one segment: of X (column
// scale 2pi sqrt(m_k)) giving G_j = (2pi)^2 sum_{k in j} m_k P_k (P_k = Re c_k^(i)
// conj c_k^(j)), and for Fejer of Y (2pi sqrt(m_k (N_j - k))) giving
// H_j = (2pi)^2 sum_{k in j} m_k (N_j - k) P_k.  Then at cutoff N = N_q
//   Dirichlet  Sigma = sum_{j<=q} G_j / (2N+1),
//   Fejer      Sigma = sum_{j<=q} ((N - N_j) G_j + H_j) / (N (N+1)),
// since the Fejer weight (1 - k/N)/(N+1) is (N - k)/(N (N+1)) and N - k =
// (N - N_j) + (N_j - k).  Every weight is >= 0, so no two separately rounded
// products are subtracted (a sum of m_k k P_k subtracted from one of m_k P_k
// cancels where the weights vanish, at small N entirely).  The reduce keeps
// sum G_j, sum N_j G_j and sum H_j in FP64 over the partials in k order.
constexpr int kSweepSegs = 64;        // distinct cutoffs of a one-pass sweep
constexpr int kSweepRanges = 128;     // k-ranges of its product
constexpr int KS = 32;                // real columns per k-step (SK and SK2)

struct SweepSeg {
    int n;                            // segments (distinct cutoffs, ascending)
    int N[kSweepSegs];
    int32_t cstart[kSweepSegs + 1];   // first column pair of each segment; cstart[n] = Kp / 2
};
struct SweepRanges {
    int nr;
    int32_t seg[kSweepRanges];        // segment of the r-th range in k order (ascending)
    int32_t part[kSweepRanges];       // its partial tile set: its place in the product's
                                      // launch order, which runs the longest ranges first
};
struct SweepSteps {
    int n;                            // entries: (first, end) k-step of each range in launch order
    int32_t v[2 * kSweepRanges];
};
struct SweepSlots {
    int n;                            // output slots (the caller's cutoffs, in their order)
    int32_t seg[kMaxCutoffs];         // segment of each slot
};

struct SweepShape {
    MfmaShape m;                      // tiles and the model's k-split
    int64_t Kp;                       // padded columns of the segment layout
    size_t xhi, xlo, yhi, ylo, p0, p1, kst, tab, total;
};

// Layout of the sweep's workspace for padded width Kp and nr ranges (bounds for
// the query: Kp <= the single-cutoff width + KS per cutoff, nr <= the model's
// split + the cutoffs).
static SweepShape sweep_shape(int32_t D, int32_t Nmax, int64_t Kp, int nr, int basis, SyrkChoice sc)
{
    SweepShape w;
    w.m = mfma_shape(D, Nmax, sc);
    w.Kp = Kp;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t op = al((size_t)w.m.Dp * Kp * 2);
    const size_t pt = al((size_t)nr * w.m.ntiles * w.m.ts * w.m.ts * 4);
    const bool fej = basis == MM_FEJER;
    size_t o = 0;
    w.xhi = o; o += op;
    w.xlo = o; o += op;
    w.yhi = o; o += fej ? op : 0;
    w.ylo = o; o += fej ? op : 0;
    w.p0 = o; o += pt;
    w.p1 = o; o += fej ? pt : 0;
    w.kst = o; o += al((size_t)2 * nr * 4);
    w.tab = o; o += al((size_t)Kp / 2 * 16);
    w.total = o;
    return w;
}

size_t cov_mfma_workspace(int32_t G, int32_t D, int32_t Nmax, SyrkChoice sc, int32_t nN)
{
    (void)G;
    size_t b = mfma_shape(D, Nmax, sc).total;
    if (nN >= 2) {
        const MfmaShape m = mfma_shape(D, Nmax, sc);
        const int n = std::min<int32_t>(nN, kSweepSegs);
        const int nr = std::min(kSweepRanges, (4 * m.nsplit + n + 7) / 8 * 8);
        b = std::max(b, sweep_shape(D, Nmax, m.Kp + (int64_t)KS * n, nr, MM_FEJER, sc).total);
    }
    return b;
}

// The column table of the segment layout, once per call: for column pair c its k
// (-1 in the padding) and the scales of X and Y (FP64, rounded to FP32); block 0
// also writes the product's k-step pairs.
__global__ void k_sweep_cols(SweepSeg seg, SweepSteps ks, int64_t kp2, int4* __restrict__ tab,
                             int32_t* __restrict__ kst)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < ks.n; i += blockDim.x) kst[i] = ks.v[i];
    if (c >= kp2) return;
    int lo = 0, hi = seg.n;                 // the last segment q with cstart[q] <= c
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg.cstart[mid] <= c) lo = mid;
        else hi = mid;
    }
    const int q = lo;
    const int k = (q == 0 ? 0 : seg.N[q - 1] + 1) + (int)(c - seg.cstart[q]);
    int4 e = make_int4(-1, 0, 0, 0);
    if (k <= seg.N[q]) {
        const double mk = k ? 2.0 : 1.0;
        e.x = k;
        e.y = __float_as_int((float)(kTwoPi * sqrt(mk)));
        e.z = __float_as_int((float)(kTwoPi * sqrt(mk * (double)(seg.N[q] - k))));
    }
    tab[c] = e;
}

// X (and for Fejer Y) of the segment layout as BF16 hi/lo pairs, from the column table.
__global__ void k_sweep_split(int D, const float2* __restrict__ coef, int64_t ldc, const int4* __restrict__ tab,
                              int64_t kp2, uint32_t* __restrict__ xhi, uint32_t* __restrict__ xlo,
                              uint32_t* __restrict__ yhi, uint32_t* __restrict__ ylo)
{
    const int64_t row = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < kp2; c += (int64_t)gridDim.x * blockDim.x) {
        const int4 e = tab[c];
        float2 cc = make_float2(0.f, 0.f);
        float s0 = 0.f, s1 = 0.f;
        if (row < D && e.x >= 0) {
            cc = coef[row * ldc + e.x];
            s0 = __int_as_float(e.y);
            s1 = __int_as_float(e.z);
        }
        uint32_t h, l;
        bf16_split_pair(cc.x, cc.y, s0, h, l);
        xhi[row * kp2 + c] = h;
        xlo[row * kp2 + c] = l;
        if (yhi) {
            bf16_split_pair(cc.x, cc.y, s1, h, l);
            yhi[row * kp2 + c] = h;
            ylo[row * kp2 + c] = l;
        }
    }
}

// The reduce of the sweep: the partial tiles of X X^T (p0, the G_j) and Y Y^T (p1,
// the H_j) added in k order in FP64 as sum G_j, sum N_j G_j and sum H_j, and at
// the end of each segment Sigma at its cutoff written, mirrored, to every output
// slot with that cutoff.  Decomposition as k_syrk_reduce.
template <int TS>
__global__ __launch_bounds__(256) void k_sweep_reduce(const float* __restrict__ p0, const float* __restrict__ p1,
                                                      SweepRanges rg, SweepSeg seg, SweepSlots sl, int basis,
                                                      int ntiles, int D, int G, int g, float* __restrict__ cov)
{
    constexpr int QN = TS / 64;
    constexpr int RB = 16;
    __shared__ float tileT[RB][65];
    const int per_tile = QN * QN * (64 / RB);
    const int t = blockIdx.x / per_tile, rem = blockIdx.x % per_tile;
    const int quad = rem / (64 / RB), part = rem % (64 / RB);
    int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (bi * (bi + 1) / 2 > t) --bi;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int qi = (quad / QN) * 64, qj = (quad % QN) * 64;
    if (bi == bj && qi < qj) return;   // mirrored from below
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t tstride = (int64_t)ntiles * TS * TS;
    const int64_t DD = (int64_t)D * D;
    double sg[RB / 4], sng[RB / 4], sh[RB / 4];   // sum G_j, sum N_j G_j, sum H_j
#pragma unroll
    for (int u = 0; u < RB / 4; ++u) sg[u] = sng[u] = sh[u] = 0.0;
    for (int r = 0; r < rg.nr; ++r) {
        const double Nj = (double)seg.N[rg.seg[r]];
#pragma unroll
        for (int u = 0; u < RB / 4; ++u) {
            const int li = qi + part * RB + ty + 4 * u, lj = qj + tx;
            const int64_t at = rg.part[r] * tstride + (int64_t)t * TS * TS + li * TS + lj;
            const double gv = (double)p0[at];
            sg[u] += gv;
            sng[u] += Nj * gv;
            if (p1) sh[u] += (double)p1[at];
        }
        if (r + 1 < rg.nr && rg.seg[r + 1] == rg.seg[r]) continue;   // uniform: the segment goes on
        const int q = rg.seg[r];
        const double Nd = (double)seg.N[q];
        float v[RB / 4];
#pragma unroll
        for (int u = 0; u < RB / 4; ++u)
            v[u] = (float)(basis == MM_DIRICHLET ? sg[u] / (2.0 * Nd + 1.0)
                                                 : (Nd * sg[u] - sng[u] + sh[u]) / (Nd * (Nd + 1.0)));
        for (int sidx = 0; sidx < sl.n; ++sidx) {
            if (sl.seg[sidx] != q) continue;   // uniform
            float* C = cov + ((int64_t)sidx * G + g) * DD;
#pragma unroll
            for (int u = 0; u < RB / 4; ++u) {
                const int lr = ty + 4 * u;
                const int i = bi * TS + qi + part * RB + lr, j = bj * TS + qj + tx;
                if (bi == bj) {
                    // diagonal tile: both entries from the lower one, so Sigma is exactly symmetric
                    if (i < D && j <= i) {
                        C[(int64_t)i * D + j] = v[u];
                        C[(int64_t)j * D + i] = v[u];
                    }
                } else {
                    if (i < D && j < D) C[(int64_t)i * D + j] = v[u];
                    tileT[lr][tx] = v[u];
                }
            }
            if (bi == bj) continue;
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * RB; e += 256) {
                const int c = e / RB, lr = e % RB;
                const int j = bj * TS + qj + c, i = bi * TS + qi + part * RB + lr;
                if (i < D && j < D) C[(int64_t)j * D + i] = tileT[lr][c];
            }
            __syncthreads();
        }
    }
}

hipError_t launch_cov_mfma_sweep(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ns, int32_t nN,
                                 int basis, void* cov, char* ws, hipStream_t st, SyrkChoice sc)
{
    // distinct cutoffs, ascending
    std::vector<int> u(Ns, Ns + nN);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    const int n = (int)u.size();
    if (n < 2 || n > kSweepSegs) return hipErrorNotSupported;
    // one pass costs one product over max N (two for Fejer); separate products cost
    // the sum of the cutoffs
    double sumN = 0.0;
    for (int v : u) sumN += (double)v + 1.0;
    if ((basis == MM_FEJER ? 2.0 : 1.0) * ((double)u.back() + 1.0) >= sumN) return hipErrorNotSupported;
    const int Nmax = u.back();
    const MfmaShape m = mfma_shape(D, Nmax, sc);
    SweepSeg seg;
    seg.n = n;
    int64_t steps = 0;
    std::vector<int64_t> seg_steps(n);
    for (int q = 0; q < n; ++q) {
        seg.N[q] = u[q];
        seg.cstart[q] = (int32_t)(steps * KS / 2);
        const int64_t cols = 2ll * (u[q] - (q ? u[q - 1] : -1));
        seg_steps[q] = (cols + KS - 1) / KS;
        steps += seg_steps[q];
    }
    seg.cstart[n] = (int32_t)(steps * KS / 2);
    const int64_t Kp = steps * KS;
    // k-ranges: each segment cut into pieces of at most about steps / (2 nsplit)
    // k-steps (half the model's single-cutoff ranges, so that the uneven pieces pack
    // evenly onto the CUs); the reduce reads them in k order
    const int64_t Lr = std::max<int64_t>(1, (steps + 4 * m.nsplit - 1) / (4 * m.nsplit));
    std::vector<int64_t> rb, re;
    std::vector<int> rq;
    int64_t at = 0;
    for (int q = 0; q < n; ++q) {
        const int64_t pieces = (seg_steps[q] + Lr - 1) / Lr;
        for (int64_t p = 0; p < pieces; ++p) {
            rb.push_back(at + seg_steps[q] * p / pieces);
            re.push_back(at + seg_steps[q] * (p + 1) / pieces);
            rq.push_back(q);
        }
        at += seg_steps[q];
    }
    const int nk = (int)rb.size();                 // ranges in k order
    const int nr = (nk + 7) / 8 * 8;               // launched: padded with empty ranges
    if (nr > kSweepRanges) return hipErrorNotSupported;
    // The product hands each XCD a contiguous eighth of its (range, tile) sequence:
    // the ranges are dealt longest first, snake-wise, into eight groups of nr/8 (equal
    // counts, near-equal k), each group in descending length, the groups in turn.
    std::vector<int> order(nk);
    for (int r = 0; r < nk; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return re[x] - rb[x] > re[y] - rb[y]; });
    std::vector<std::vector<int>> grp(8);
    for (int i = 0; i < nr; ++i) {
        const int round = i / 8, pos = i % 8;
        grp[round & 1 ? 7 - pos : pos].push_back(i < nk ? order[i] : -1);
    }
    SweepRanges rg;
    SweepSteps ks;
    rg.nr = nk;
    ks.n = 2 * nr;
    int s2 = 0;
    for (int x = 0; x < 8; ++x)
        for (int r : grp[x]) {
            ks.v[2 * s2] = r < 0 ? 0 : (int32_t)rb[r];
            ks.v[2 * s2 + 1] = r < 0 ? 0 : (int32_t)re[r];
            if (r >= 0) rg.part[r] = s2;
            ++s2;
        }
    for (int r = 0; r < nk; ++r) rg.seg[r] = rq[r];
    SweepSlots sl;
    sl.n = nN;
    for (int i = 0; i < nN; ++i) sl.seg[i] = (int32_t)(std::lower_bound(u.begin(), u.end(), Ns[i]) - u.begin());
    const SweepShape w = sweep_shape(D, Nmax, Kp, nr, basis, sc);
    if (w.total > cov_mfma_workspace(G, D, Nmax, sc, nN)) return hipErrorNotSupported;   // outside the queried bound
    const bool fej = basis == MM_FEJER;
    uint16_t* xhi = (uint16_t*)(ws + w.xhi);
    uint16_t* xlo = (uint16_t*)(ws + w.xlo);
    uint16_t* yhi = fej ? (uint16_t*)(ws + w.yhi) : nullptr;
    uint16_t* ylo = fej ? (uint16_t*)(ws + w.ylo) : nullptr;
    float* p0 = (float*)(ws + w.p0);
    float* p1 = fej ? (float*)(ws + w.p1) : nullptr;
    int32_t* kst = (int32_t*)(ws + w.kst);
    int4* tab = (int4*)(ws + w.tab);
    prof_begin("k_sweep_cols", st);
    hipLaunchKernelGGL(k_sweep_cols, dim3((unsigned)((Kp / 2 + 255) / 256)), dim3(256), 0, st, seg, ks, Kp / 2, tab,
                       kst);
    prof_end("k_sweep_cols", st);
    for (int g = 0; g < G; ++g) {
        const float2* cg = (const float2*)coef + (int64_t)g * D * ldc;
        const int bx = (int)std::min<int64_t>((Kp / 2 + 255) / 256, 64);
        prof_begin("k_sweep_split", st);
        hipLaunchKernelGGL(k_sweep_split, dim3(bx, m.Dp), dim3(256), 0, st, D, cg, ldc, (const int4*)tab, Kp / 2,
                           (uint32_t*)xhi, (uint32_t*)xlo, (uint32_t*)yhi, (uint32_t*)ylo);
        prof_end("k_sweep_split", st);
        const char* name = m.ts == T2 ? "k_syrk_mfma256" : "k_syrk_mfma";
        for (int pass = 0; pass < (fej ? 2 : 1); ++pass) {
            const uint16_t* ah = pass ? yhi : xhi;
            const uint16_t* al = pass ? ylo : xlo;
            float* pp = pass ? p1 : p0;
            prof_begin(name, st);
            if (m.ts == T2)
                hipLaunchKernelGGL(k_syrk_mfma256, dim3((unsigned)(m.ntiles * nr)), dim3(256), 0, st, ah, al, ah, al,
                                   Kp, (int64_t)0, m.ntiles, nr, pp, (const int32_t*)kst);
            else
                hipLaunchKernelGGL(k_syrk_mfma, dim3((unsigned)(m.ntiles * nr)), dim3(256), 0, st, ah, al, ah, al,
                                   Kp, (int64_t)0, m.ntiles, nr, pp, (const int32_t*)kst);
            prof_end(name, st);
        }
        prof_begin("k_sweep_reduce", st);
        if (m.ts == T2)
            hipLaunchKernelGGL(k_sweep_reduce<T2>, dim3((unsigned)(64 * m.ntiles)), dim3(256), 0, st, p0, p1, rg, seg,
                               sl, basis, m.ntiles, D, G, g, (float*)cov);
        else
            hipLaunchKernelGGL(k_sweep_reduce<ST>, dim3((unsigned)(16 * m.ntiles)), dim3(256), 0, st, p0, p1, rg, seg,
                               sl, basis, m.ntiles, D, G, g, (float*)cov);
        prof_end("k_sweep_reduce", st);
    }
    return hipGetLastError();
}

// Zero padding of the split operands when the row pass writes them: the pairs
// from column ncol on of rows below D (tail = kp2 - ncol each), then rows
// D..Dp-1 whole, as one grid-stride range.
__global__ void k_split_pad(int D, int Dp, int64_t ncol, int64_t kp2, uint32_t* __restrict__ hi,
                            uint32_t* __restrict__ lo)
{
    const int64_t tail = kp2 - ncol;
    const int64_t n1 = (int64_t)D * tail, total = n1 + (int64_t)(Dp - D) * kp2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t at = i < n1 ? (i / tail) * kp2 + ncol + i % tail : (int64_t)D * kp2 + (i - n1);
        hi[at] = 0u;
        lo[at] = 0u;
    }
}

int32_t split_out_cols(int32_t N, int32_t L1) { return L1 * ((N + L1) / L1); }

SplitOut cov_mfma_split_out(int32_t D, int32_t N, int32_t L1, char* ws, SyrkChoice sc)
{
    const int32_t ncol = split_out_cols(N, L1);
    const MfmaShape s = mfma_shape(D, ncol - 1, sc);
    SplitOut o;
    o.hi = (uint32_t*)(ws + s.hi);
    o.lo = (uint32_t*)(ws + s.lo);
    o.kp2 = s.Kp / 2;
    o.k2n = ncol / L1;
    o.scale = (const float*)(ws + s.scale);
    o.fac = (float*)(ws + s.fac);
    return o;
}

hipError_t launch_split_prologue(int32_t D, int32_t N, int32_t L1, int basis, char* ws, hipStream_t st,
                                 SyrkChoice sc)
{
    const int32_t ncol = split_out_cols(N, L1);
    const MfmaShape s = mfma_shape(D, ncol - 1, sc);
    prof_begin("k_split_scale", st);
    hipLaunchKernelGGL(k_split_scale, dim3((unsigned)((s.Kp / 2 + 255) / 256)), dim3(256), 0, st, N, basis, s.Kp / 2,
                       (float*)(ws + s.scale));
    prof_end("k_split_scale", st);
    const int64_t kp2 = s.Kp / 2;
    const int64_t total = (int64_t)D * (kp2 - ncol) + (s.Dp - D) * kp2;
    const int bx = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1024));
    prof_begin("k_split_pad", st);
    hipLaunchKernelGGL(k_split_pad, dim3(bx), dim3(256), 0, st, D, (int)s.Dp, (int64_t)ncol, kp2,
                       (uint32_t*)(ws + s.hi), (uint32_t*)(ws + s.lo));
    prof_end("k_split_pad", st);
    return hipGetLastError();
}

// Workspace of the one-pass per-pair product (after the caller's tables): the
// variance table, then (MM_MIXED) the A and B operands and the split-K partials.
struct PairShape {
    MfmaShape m;
    size_t var, bhi, blo, mfma, total;
};

static PairShape pair_shape(int prec, int32_t G, int32_t D, int32_t Nmax, int32_t nq)
{
    PairShape s;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t es = prec == MM_MIXED ? 4 : 8;
    s.var = 0;
    size_t o = al((size_t)G * D * nq * es);
    if (prec == MM_MIXED) {
        s.m = mfma_shape(D, Nmax);
        s.bhi = o; o += al((size_t)s.m.Dp * s.m.Kp * 2);
        s.blo = o; o += al((size_t)s.m.Dp * s.m.Kp * 2);
        s.mfma = o; o += s.m.total;
    } else {
        s.bhi = s.blo = s.mfma = o;
    }
    s.total = o;
    return s;
}

size_t cov_pair_workspace(int prec, int32_t G, int32_t D, int32_t Nmax, int32_t nq)
{
    return pair_shape(prec, G, D, Nmax, nq).total;
}

hipError_t launch_cov_pair(int prec, int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t Nmax,
                           const PairTables& tb, int32_t nq, int basis, void* cov, void* corr, char* ws,
                           hipStream_t st)
{
    const PairShape s = pair_shape(prec, G, D, Nmax, nq);
    const size_t es = prec == MM_MIXED ? 4 : 8;
    for (int g = 0; g < G; ++g) {
        char* cg = (char*)cov + (size_t)g * D * D * es;
        if (prec == MM_MIXED) {
            const MfmaShape& m = s.m;
            char* w = ws + s.mfma;
            uint16_t* ahi = (uint16_t*)(w + m.hi);
            uint16_t* alo = (uint16_t*)(w + m.lo);
            uint16_t* bhi = (uint16_t*)(ws + s.bhi);
            uint16_t* blo = (uint16_t*)(ws + s.blo);
            float* part = (float*)(w + m.partial);
            const int bx = (int)std::min<int64_t>((m.Kp / 2 + 255) / 256, 64);
            prof_begin("k_pair_split", st);
            hipLaunchKernelGGL(k_pair_split, dim3(bx, m.Dp), dim3(256), 0, st, D,
                               (const float2*)coef + (int64_t)g * D * ldc, ldc, tb.perm, tb.Nr, basis, m.Kp,
                               (uint32_t*)ahi, (uint32_t*)alo, (uint32_t*)bhi, (uint32_t*)blo);
            prof_end("k_pair_split", st);
            const char* name = m.ts == T2 ? "k_syrk_mfma256" : "k_syrk_mfma";
            prof_begin(name, st);
            if (m.ts == T2)
                hipLaunchKernelGGL(k_syrk_mfma256, dim3((unsigned)(m.ntiles * m.nsplit)), dim3(256), 0, st, ahi, alo,
                                   bhi, blo, m.Kp, m.kchunk, m.ntiles, m.nsplit, part, (const int32_t*)nullptr);
            else
                hipLaunchKernelGGL(k_syrk_mfma, dim3((unsigned)(m.ntiles * m.nsplit)), dim3(256), 0, st, ahi, alo,
                                   bhi, blo, m.Kp, m.kchunk, m.ntiles, m.nsplit, part, (const int32_t*)nullptr);
            prof_end(name, st);
            prof_begin("k_syrk_reduce", st);
            if (m.ts == T2)
                hipLaunchKernelGGL(k_syrk_reduce<T2>, dim3((unsigned)(64 * m.ntiles)), dim3(256), 0, st, part,
                                   m.nsplit, m.ntiles, D, (float*)cg, tb.perm);
            else
                hipLaunchKernelGGL(k_syrk_reduce<ST>, dim3((unsigned)(16 * m.ntiles)), dim3(256), 0, st, part,
                                   m.nsplit, m.ntiles, D, (float*)cg, tb.perm);
            prof_end("k_syrk_reduce", st);
        } else {
            const int tn = (D + F64T - 1) / F64T;
            prof_begin("k_pair_fp64", st);
            hipLaunchKernelGGL(k_pair_fp64, dim3(tn * (tn + 1) / 2), dim3(256), 0, st, D,
                               (const double2*)coef + (int64_t)g * D * ldc, ldc, Nmax, tb.perm, tb.Nr, basis,
                               (double*)cg);
            prof_end("k_pair_fp64", st);
        }
    }
    if (corr) {
        prof_begin("k_pair_var", st);
        if (prec == MM_MIXED)
            hipLaunchKernelGGL((k_pair_var<float2, float>), dim3(D, G), dim3(64), 0, st, D, (const float2*)coef, ldc,
                               tb.perm, tb.Nr, tb.cutq, nq, basis, (float*)(ws + s.var));
        else
            hipLaunchKernelGGL((k_pair_var<double2, double>), dim3(D, G), dim3(64), 0, st, D, (const double2*)coef,
                               ldc, tb.perm, tb.Nr, tb.cutq, nq, basis, (double*)(ws + s.var));
        prof_end("k_pair_var", st);
        const int64_t total = (int64_t)G * D * D;
        const int blocks = (int)((total + 255) / 256);
        prof_begin("k_pair_corr", st);
        if (prec == MM_MIXED)
            hipLaunchKernelGGL(k_pair_corr<float>, dim3(blocks), dim3(256), 0, st, total, D, tb.rank, tb.slot,
                               (const float*)(ws + s.var), nq, (const float*)cov, (float*)corr);
        else
            hipLaunchKernelGGL(k_pair_corr<double>, dim3(blocks), dim3(256), 0, st, total, D, tb.rank, tb.slot,
                               (const double*)(ws + s.var), nq, (const double*)cov, (double*)corr);
        prof_end("k_pair_corr", st);
    }
    return hipGetLastError();
}

hipError_t launch_cov_mfma(int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t N, int basis, void* cov,
                           char* ws, hipStream_t st, bool operands_ready, SyrkChoice sc)
{
    MfmaShape s = mfma_shape(D, N, sc);
    uint16_t* hi = (uint16_t*)(ws + s.hi);
    uint16_t* lo = (uint16_t*)(ws + s.lo);
    float* part = (float*)(ws + s.partial);
    float* scale = (float*)(ws + s.scale);
    if (operands_ready && G != 1) return hipErrorInvalidValue;
    if (!operands_ready) {
        prof_begin("k_split_scale", st);
        hipLaunchKernelGGL(k_split_scale, dim3((unsigned)((s.Kp / 2 + 255) / 256)), dim3(256), 0, st, N, basis,
                           s.Kp / 2, scale);
        prof_end("k_split_scale", st);
    }
    for (int g = 0; g < G; ++g) {
        const float2* cg = (const float2*)coef + (int64_t)g * D * ldc;
        int bx = (int)std::min<int64_t>((s.Kp / 2 + 255) / 256, 64);
        if (!operands_ready) {
            prof_begin("k_split_bf16", st);
            hipLaunchKernelGGL(k_split_bf16, dim3(bx, s.Dp), dim3(256), 0, st, D, cg, ldc, N, (const float*)scale,
                               s.Kp, hi, lo);
            prof_end("k_split_bf16", st);
        }
        const char* syrk_name = s.ts == T2 ? "k_syrk_mfma256" : "k_syrk_mfma";
        prof_begin(syrk_name, st);
        if (s.ts == T2)
            hipLaunchKernelGGL(k_syrk_mfma256, dim3((unsigned)(s.ntiles * s.nsplit)), dim3(256), 0, st, hi, lo, hi, lo,
                               s.Kp, s.kchunk, s.ntiles, s.nsplit, part, (const int32_t*)nullptr);
        else
            hipLaunchKernelGGL(k_syrk_mfma, dim3((unsigned)(s.ntiles * s.nsplit)), dim3(256), 0, st, hi, lo, hi, lo,
                               s.Kp, s.kchunk, s.ntiles, s.nsplit, part, (const int32_t*)nullptr);
        prof_end(syrk_name, st);
        prof_begin("k_syrk_reduce", st);
        if (s.ts == T2)
            hipLaunchKernelGGL(k_syrk_reduce<T2>, dim3((unsigned)(64 * s.ntiles)), dim3(256), 0, st, part, s.nsplit,
                               s.ntiles, D, (float*)cov + (int64_t)g * D * D, (const int32_t*)nullptr);
        else
            hipLaunchKernelGGL(k_syrk_reduce<ST>, dim3((unsigned)(16 * s.ntiles)), dim3(256), 0, st, part, s.nsplit,
                               s.ntiles, D, (float*)cov + (int64_t)g * D * D, (const int32_t*)nullptr);
        prof_end("k_syrk_reduce", st);
    }
    return hipGetLastError();
}

}  // namespace mm
