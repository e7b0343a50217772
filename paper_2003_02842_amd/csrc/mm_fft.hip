// Grid FFT of the type-1 NUFFT (Eq. Der:16) with one LDS exchange per pass.
//
// The packed complex grid z_j = x_2j + i x_2j+1 (length L = Mr/2 = L1 L2) is an
// L1 x L2 row-major matrix (rows L2p apart).  Both passes split their
// sub-transform of length n = A B by Cooley-Tukey, with n = B n_a + n_b and
// k = k_a + A k_b:
//   X[k_a + A k_b] = sum_{n_b} W_B^{n_b k_b} W_n^{n_b k_a} sum_{n_a} x[B n_a + n_b] W_A^{n_a k_a}
// Step A (size-A DFTs) runs on values a thread loads straight from HBM, the
// product with W_n^{n_b k_a} follows, one LDS exchange regroups the values, and
// step B (size-B DFTs) leaves every output in natural order.  Both DFT sizes are
// 2,3,5-smooth and at most 32; each is a fully unrolled register codelet with
// compile-time twiddles.
//
//   k_fft_cols_ab  length-L1 transforms of the columns, times the four-step
//                  twiddle W_L^{k1 l2}, in place
//   k_fft_rows_ab  length-L2 transforms of the row pairs (k1, L1 - k1), the
//                  real-input untangling, deconvolution (Eq. Der:17) and the 1/2pi
//                  of the coefficient definition; writes c_k, k = 0..N, or (the
//                  split step fused) the contraction's BF16 operands, one
//                  contiguous run per row
//
// Long twiddle tables are split in two, W^m = lo[m mod LO] hi[m / LO], so both
// halves (about 2 sqrt(L) entries) sit in LDS.
#include <hip/hip_runtime.h>

#include "mm_bf16.h"
#include "mm_fft_codelets.h"
#include "mm_internal.h"

#ifndef MM_FFT_ROWS_XCD
#define MM_FFT_ROWS_XCD 1
#endif

namespace mm {

// Workgroup (column block, series): CC consecutive columns, each transformed by
// B threads in step A and A threads in step B.  LDS: tw1 (L1), the split W_L
// table, then A blocks of B*CC values (one pad value per block).
template <typename T>
__global__ __launch_bounds__(512) void k_fft_cols_ab(T* __restrict__ grid, int64_t grid_stride, int L1, int L2,
                                                     int L2p, int A, int B, int CC,
                                                     const typename CTf<T>::type* __restrict__ tw1g,
                                                     const typename CTf<T>::type* __restrict__ log_,
                                                     const typename CTf<T>::type* __restrict__ hig, int lo_bits,
                                                     int n_hi)
{
    using C = typename CTf<T>::type;
    extern __shared__ __align__(16) char smem_raw[];
    C* tw1 = reinterpret_cast<C*>(smem_raw);
    C* lo = tw1 + L1;
    C* hi = lo + (1 << lo_bits);
    C* sh = hi + n_hi;
    const int blk = B * CC + 1;
    for (int i = threadIdx.x; i < L1; i += blockDim.x) tw1[i] = tw1g[i];
    for (int i = threadIdx.x; i < (1 << lo_bits); i += blockDim.x) lo[i] = log_[i];
    for (int i = threadIdx.x; i < n_hi; i += blockDim.x) hi[i] = hig[i];
    C* z = reinterpret_cast<C*>(grid + (int64_t)blockIdx.y * grid_stride);
    const int c0 = blockIdx.x * CC;
    const int c = (int)threadIdx.x % CC, r = (int)threadIdx.x / CC;
    const int col = c0 + c;
    __syncthreads();
    if (r < B && col < L2) {
        switch (A) {
#define MM_CASE_A(n) case n: col_step_a<T, n>(z, L2p, B, r, col, tw1, sh, blk, r * CC + c); break;
            MM_CODELETS(MM_CASE_A)
#undef MM_CASE_A
        }
    }
    __syncthreads();
    if (r < A && col < L2) {
        switch (B) {
#define MM_CASE_B(n) case n: col_step_b<T, n>(z, L2p, A, r, col, CC, sh, blk, c, lo, hi, lo_bits); break;
            MM_CODELETS(MM_CASE_B)
#undef MM_CASE_B
        }
    }
}

// Workgroup (row-pair block, series): rows k1 = p0 + i and their mirrors
// (L1 - k1) mod L1 for i < RR, then for k = k1 + L1 k2 <= N
//   X_k = (Z_k + conj Z_{L-k})/2 - (i/2) W_Mr^k (Z_k - conj Z_{L-k})
// (Z_{L-k} sits in the mirror row at column L2-1-k2, or (L2-k2) mod L2 when
// k1 = 0), times the deconvolution factor.  LDS: tw2 (L2), the split W_Mr
// table, then 2 RR rows of L2 + 1 values.
template <typename T>
__global__ __launch_bounds__(512) void k_fft_rows_ab(const T* __restrict__ grid, int64_t grid_stride, int L1,
                                                     int L2, int L2p, int A, int B, int RR,
                                                     const typename CTf<T>::type* __restrict__ tw2g,
                                                     const typename CTf<T>::type* __restrict__ log_,
                                                     const typename CTf<T>::type* __restrict__ hig, int lo_bits,
                                                     int n_hi, const T* __restrict__ dfac, int N,
                                                     typename CTf<T>::type* __restrict__ coef, int64_t ldc, int s_out,
                                                     SplitOut so)
{
    using C = typename CTf<T>::type;
    extern __shared__ __align__(16) char smem_raw[];
    C* tw2 = reinterpret_cast<C*>(smem_raw);
    C* lo = tw2 + L2;
    C* hi = lo + (1 << lo_bits);
    C* sh = hi + n_hi;
    const int rs = L2 + 1;
    for (int i = threadIdx.x; i < L2; i += blockDim.x) tw2[i] = tw2g[i];
    for (int i = threadIdx.x; i < (1 << lo_bits); i += blockDim.x) lo[i] = log_[i];
    for (int i = threadIdx.x; i < n_hi; i += blockDim.x) hi[i] = hig[i];
    // Work item (row block bx, series by).  Writing c_k, in an XCD-aware order:
    // workgroups are dealt to the eight XCDs in turn, and each XCD takes a
    // contiguous run of the row-block-major sequence, so that the row blocks whose
    // outputs share 128-byte lines (k = k1 + L1 k2 with consecutive k1) are written
    // through one L2 at about the same time rather than as partial lines from
    // several.  The fused split writes whole rows and keeps the launch order
    // (0.54 vs 0.59 ms on a 155,520-cell grid).
    int bx = (int)blockIdx.x, by = (int)blockIdx.y;
    if (MM_FFT_ROWS_XCD && !so.hi) {
        const int nwg = (int)(gridDim.x * gridDim.y);
        const int lin = (int)(blockIdx.x + gridDim.x * blockIdx.y);
        const int per = nwg >> 3, rem = nwg & 7, x = lin & 7, r = lin >> 3;
        const int w = x * per + min(x, rem) + r;
        bx = w % (int)gridDim.x;
        by = w / (int)gridDim.x;
    }
    const C* Y = reinterpret_cast<const C*>(grid + (int64_t)by * grid_stride);
    C* out = coef + (int64_t)(s_out + by) * ldc;
    const int P = L1 / 2 + 1;
    const int p0 = bx * RR;
    const int nr = min(RR, P - p0);
    // LDS row 2i: matrix row p0 + i; row 2i + 1: its mirror
    auto mrow = [&](int r) { const int p = p0 + (r >> 1); return (r & 1) ? (L1 - p) % L1 : p; };
    __syncthreads();
    {
        const int nb = (int)threadIdx.x % B, r = (int)threadIdx.x / B;
        if (r < 2 * nr) {
            const C* row = Y + (int64_t)mrow(r) * L2p;
            switch (A) {
#define MM_CASE_A(n) case n: row_step_a<T, n>(row, B, nb, tw2, sh + r * rs); break;
                MM_CODELETS(MM_CASE_A)
#undef MM_CASE_A
            }
        }
    }
    __syncthreads();
    {
        const int ka = (int)threadIdx.x % A, r = (int)threadIdx.x / A;
        C y[32];
        const bool act = r < 2 * nr;
        if (act) {
            switch (B) {
#define MM_CASE_B(n) case n: row_step_b<T, n>(sh + r * rs, ka, y); break;
                MM_CODELETS(MM_CASE_B)
#undef MM_CASE_B
            }
        }
        __syncthreads();
        if (act) {
            switch (B) {
#define MM_CASE_S(n) case n: row_store_b<T, n>(sh + r * rs, A, ka, y); break;
                MM_CODELETS(MM_CASE_S)
#undef MM_CASE_S
            }
        }
    }
    __syncthreads();
    // X_k for rows k1 and columns k2 (Zk: row k1, column k2; Zm: the mirror value)
    auto untangle = [&](int i, int side, int k1, int k2, int k, C& A, C& WB) {
        const int k2m = (k1 == 0) ? (k2 == 0 ? 0 : L2 - k2) : (L2 - 1 - k2);
        const C Zk = sh[(2 * i + side) * rs + k2];
        const C Zm = sh[(2 * i + 1 - side) * rs + k2m];
        A = C{Zk.x + Zm.x, Zk.y - Zm.y};
        const C Bv = C{Zk.x - Zm.x, Zk.y + Zm.y};
        WB = cmulf(tw_split(lo, hi, k, lo_bits), Bv);
    };
    if constexpr (sizeof(T) == 4) {
        if (so.hi) {
            // the split step fused (SplitOut): row k1's coefficients k = k1 + L1 k2 go to
            // columns k1 K2 + k2 of the operand row, so each row is one contiguous run;
            // X = (s_k d_k / 2) (A + ...), the factor from the set-up's table (zero where
            // k > N), as BF16 hi and lo
            const int K2 = so.k2n;
            uint32_t* const hrow = so.hi + (int64_t)(s_out + by) * so.kp2;
            uint32_t* const lrow = so.lo + (int64_t)(s_out + by) * so.kp2;
            for (int r = 0; r < 2 * nr; ++r) {
                const int i = r >> 1, side = r & 1;
                const int p = p0 + i;
                const int rowA = p, rowB = (L1 - p) % L1;
                if (side && rowB == rowA) continue;
                const int k1 = side ? rowB : rowA;
                const int64_t c0 = (int64_t)k1 * K2;
                for (int k2 = threadIdx.x; k2 < K2; k2 += blockDim.x) {
                    C A, WB;
                    untangle(i, side, k1, k2, k1 + L1 * k2, A, WB);
                    uint32_t h, l;
                    bf16_split_pair(A.x + WB.y, A.y - WB.x, so.fac[c0 + k2], h, l);
                    hrow[c0 + k2] = h;
                    lrow[c0 + k2] = l;
                }
            }
            return;
        }
    }
    // RR is a power of two: row index fastest, so R consecutive k share a segment.
    // Only columns k2 <= (N - p0)/L1 can hold a k <= N.
    const int rr_bits = __ffs(RR) - 1;
    const int K2 = min(L2, (N - p0) / L1 + 1);
    const int total = 2 * RR * K2;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int i = idx & (RR - 1);
        const int t2 = idx >> rr_bits;
        const int side = t2 & 1, k2 = t2 >> 1;
        const int p = p0 + i;
        if (i >= nr) continue;
        const int rowA = p, rowB = (L1 - p) % L1;
        if (side && rowB == rowA) continue;
        const int k1 = side ? rowB : rowA;
        const int64_t k = (int64_t)k1 + (int64_t)L1 * k2;
        if (k > N) continue;
        C Av, WB;
        untangle(i, side, k1, k2, (int)k, Av, WB);
        const T d = dfac[k] * (T)0.5;
        out[k] = C{(Av.x + WB.y) * d, (Av.y - WB.x) * d};
    }
}

// FP64 tables of the two passes (fft_tables_at), one entry per thread.
template <typename T>
__global__ void k_fft_tables(FftTables<T> b)
{
    fft_tables_at<T>(b, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- host side
static int round64(int x) { return (x + 63) & ~63; }

template <typename T>
static hipError_t fft_ab_t(const Plan& p, const NufftWs& w, char* ws, int32_t s_begin, int32_t s_count, T* grid,
                           int64_t gstride, void* coef, int64_t ldc, hipStream_t st, const SplitOut* so)
{
    const SplitOut none{};
    using C = typename CTf<T>::type;
    const int t1 = round64(p.CC * std::max(p.A1, p.B1));
    prof_begin("k_fft_cols_ab", st);
    hipLaunchKernelGGL(k_fft_cols_ab<T>, dim3((p.L2 + p.CC - 1) / p.CC, s_count), dim3(t1), fft_ab_lds_cols(p), st,
                       grid, gstride, p.L1, p.L2, p.L2p, p.A1, p.B1, p.CC, (const C*)(ws + w.tw1),
                       (const C*)(ws + w.tLlo), (const C*)(ws + w.tLhi), p.tw_lo_bits, p.tw_hi_L);
    prof_end("k_fft_cols_ab", st);
    const int P = p.L1 / 2 + 1;
    const int t2 = round64(std::max(2 * p.RR * std::max(p.A2, p.B2), 64));
    prof_begin("k_fft_rows_ab", st);
    hipLaunchKernelGGL(k_fft_rows_ab<T>, dim3((P + p.RR - 1) / p.RR, s_count), dim3(t2), fft_ab_lds_rows(p), st,
                       grid, gstride, p.L1, p.L2, p.L2p, p.A2, p.B2, p.RR, (const C*)(ws + w.tw2),
                       (const C*)(ws + w.tMlo), (const C*)(ws + w.tMhi), p.tw_lo_bits, p.tw_hi_M,
                       (const T*)(ws + w.dfac), p.N, (C*)coef, ldc, s_begin, so ? *so : none);
    prof_end("k_fft_rows_ab", st);
    return hipGetLastError();
}

hipError_t launch_fft_ab(const Plan& p, const NufftWs& w, char* ws, int32_t s_begin, int32_t s_count, void* grid,
                         int64_t gstride, void* coef, int64_t ldc, hipStream_t st, const SplitOut* so)
{
    if (p.prec == MM_MIXED)
        return fft_ab_t<float>(p, w, ws, s_begin, s_count, (float*)grid, gstride, coef, ldc, st, so);
    if (so) return hipErrorInvalidValue;
    return fft_ab_t<double>(p, w, ws, s_begin, s_count, (double*)grid, gstride, coef, ldc, st, nullptr);
}

hipError_t launch_fft_ab_tables(const Plan& p, const NufftWs& w, char* ws, hipStream_t st)
{
    const int blocks = (int)((fft_tables_count(p) + 255) / 256);
    if (p.prec == MM_MIXED)
        hipLaunchKernelGGL(k_fft_tables<float>, dim3(blocks), dim3(256), 0, st, fft_tables_of<float>(p, w, ws));
    else
        hipLaunchKernelGGL(k_fft_tables<double>, dim3(blocks), dim3(256), 0, st, fft_tables_of<double>(p, w, ws));
    return hipGetLastError();
}

}  // namespace mm
