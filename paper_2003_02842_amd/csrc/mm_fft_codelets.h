// Register codelets and the steps of the two-pass grid FFT (Eq. Der:16), shared
// by the HBM-resident passes (mm_fft.hip) and the fused small-grid NUFFT, whose
// grid stays in LDS (mm_fused.hip).  Device code only.
//
// A sub-transform of length n = A B splits by Cooley-Tukey with n = B n_a + n_b,
// k = k_a + A k_b:
//   X[k_a + A k_b] = sum_{n_b} W_B^{n_b k_b} W_n^{n_b k_a} sum_{n_a} x[B n_a + n_b] W_A^{n_a k_a}
// Step A (size-A DFTs) runs on values a thread loads, the product with
// W_n^{n_b k_a} follows, one exchange through LDS regroups the values, and step B
// (size-B DFTs) leaves every output in natural order.  Both DFT sizes are
// 2,3,5-smooth and at most 32; each is a fully unrolled register codelet with
// compile-time twiddles.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mm_internal.h"

namespace mm {

template <typename T> struct CTf;
template <> struct CTf<float> { using type = float2; };
template <> struct CTf<double> { using type = double2; };

// Twiddle tables of the two-pass FFT (FP64 sincospi, rounded to T): W_L1^j,
// W_L2^j, and the split tables W_L^m, W_Mr^m = lo[m mod 2^lo_bits] hi[m >> lo_bits].
template <typename T>
struct FftTables {
    int L1, L2, L, Mr, lo_bits, n_hi_L, n_hi_M;
    typename CTf<T>::type *tw1, *tw2, *Llo, *Lhi, *Mlo, *Mhi;
};
template <typename T>
inline FftTables<T> fft_tables_of(const Plan& p, const NufftWs& w, char* ws)
{
    using C = typename CTf<T>::type;
    return FftTables<T>{p.L1, p.L2, p.L, p.Mr, p.tw_lo_bits, p.tw_hi_L, p.tw_hi_M, (C*)(ws + w.tw1), (C*)(ws + w.tw2),
                        (C*)(ws + w.tLlo), (C*)(ws + w.tLhi), (C*)(ws + w.tMlo), (C*)(ws + w.tMhi)};
}
// entries in order: L1, L2, 2^lo_bits (both lo tables), n_hi_L, n_hi_M
inline int64_t fft_tables_count(const Plan& p)
{
    return (int64_t)p.L1 + p.L2 + (1 << p.tw_lo_bits) + p.tw_hi_L + p.tw_hi_M;
}
template <typename T>
__device__ __forceinline__ void fft_tables_at(const FftTables<T>& b, int64_t i)
{
    using C = typename CTf<T>::type;
    auto tw = [](int64_t j, int64_t n) {
        double s, c;
        sincospi(2.0 * (double)(j % n) / (double)n, &s, &c);
        return C{(T)c, (T)-s};
    };
    const int LO = 1 << b.lo_bits;
    if (i < b.L1) { b.tw1[i] = tw(i, b.L1); return; }
    i -= b.L1;
    if (i < b.L2) { b.tw2[i] = tw(i, b.L2); return; }
    i -= b.L2;
    if (i < LO) { b.Llo[i] = tw(i, b.L); b.Mlo[i] = tw(i, b.Mr); return; }
    i -= LO;
    if (i < b.n_hi_L) { b.Lhi[i] = tw(i * LO, b.L); return; }
    i -= b.n_hi_L;
    if (i < b.n_hi_M) { b.Mhi[i] = tw(i * LO, b.Mr); return; }
}

// ---------------------------------------------------------------- compile-time twiddles
// cos and sin of 2 pi m / n by octant reduction and Taylor series (|x| <= pi/4).
__host__ __device__ constexpr double cx_sin_t(double x)
{
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
__host__ __device__ constexpr double cx_cos_t(double x)
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// cos(2 pi f) for f in [0, 1/4]
__host__ __device__ constexpr double cx_cos_q(double f)
{
    constexpr double pi = 3.141592653589793238462643383279502884;
    return f <= 0.125 ? cx_cos_t(2.0 * pi * f) : cx_sin_t(2.0 * pi * (0.25 - f));
}
__host__ __device__ constexpr double cx_cos2pi(int m, int n)
{
    m %= n;
    if (m < 0) m += n;
    double f = (double)m / (double)n;
    if (f > 0.5) f = 1.0 - f;                       // cos even about 1/2
    return f > 0.25 ? -cx_cos_q(0.5 - f) : cx_cos_q(f);
}
__host__ __device__ constexpr double cx_sin2pi(int m, int n)
{
    // sin(2 pi m/n) = cos(2 pi (m/n - 1/4)) = cos(2 pi (4m - n) / 4n)
    return cx_cos2pi(4 * (m % n) - n, 4 * n);
}

// cos and sin of 2 pi m / N, m < N, evaluated by the compiler.
template <int N>
struct TwTable {
    double c[N], s[N];
    constexpr TwTable() : c(), s()
    {
        for (int m = 0; m < N; ++m) {
            c[m] = cx_cos2pi(m, N);
            s[m] = cx_sin2pi(m, N);
        }
    }
};
template <int N>
struct TwConst {
    static constexpr TwTable<N> tab{};
};

// v * W_N^m = v exp(-2 pi i m / N); m is a constant once the codelet loops unroll.
template <typename T, int N>
__device__ __forceinline__ typename CTf<T>::type twc(typename CTf<T>::type v, int m)
{
    using C = typename CTf<T>::type;
    m %= N;
    if (m == 0) return v;
    if (4 * m == N) return C{v.y, -v.x};
    if (2 * m == N) return C{-v.x, -v.y};
    if (4 * m == 3 * N) return C{-v.y, v.x};
    const T c = (T)TwConst<N>::tab.c[m], s = (T)TwConst<N>::tab.s[m];
    return C{fma(v.x, c, v.y * s), fma(v.y, c, -(v.x * s))};
}

// ---------------------------------------------------------------- register codelets
// In-place forward DFT of R <= 5 values, exp(-2 pi i/R).
template <typename T, int R>
__device__ __forceinline__ void dft_small(typename CTf<T>::type* v)
{
    using C = typename CTf<T>::type;
    if constexpr (R == 2) {
        C a = v[0], b = v[1];
        v[0] = C{a.x + b.x, a.y + b.y};
        v[1] = C{a.x - b.x, a.y - b.y};
    } else if constexpr (R == 3) {
        const T s3 = (T)0.86602540378443864676;
        C t1 = C{v[1].x + v[2].x, v[1].y + v[2].y};
        C t2 = C{v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
        C t3 = C{s3 * (v[1].x - v[2].x), s3 * (v[1].y - v[2].y)};
        v[0] = C{v[0].x + t1.x, v[0].y + t1.y};
        v[1] = C{t2.x + t3.y, t2.y - t3.x};
        v[2] = C{t2.x - t3.y, t2.y + t3.x};
    } else if constexpr (R == 4) {
        C a = C{v[0].x + v[2].x, v[0].y + v[2].y}, b = C{v[0].x - v[2].x, v[0].y - v[2].y};
        C c = C{v[1].x + v[3].x, v[1].y + v[3].y}, d = C{v[1].x - v[3].x, v[1].y - v[3].y};
        v[0] = C{a.x + c.x, a.y + c.y};
        v[2] = C{a.x - c.x, a.y - c.y};
        v[1] = C{b.x + d.y, b.y - d.x};
        v[3] = C{b.x - d.y, b.y + d.x};
    } else if constexpr (R == 5) {
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        C x0 = v[0];
        C a1 = C{v[1].x + v[4].x, v[1].y + v[4].y}, b1 = C{v[1].x - v[4].x, v[1].y - v[4].y};
        C a2 = C{v[2].x + v[3].x, v[2].y + v[3].y}, b2 = C{v[2].x - v[3].x, v[2].y - v[3].y};
        C p1 = C{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
        C q1 = C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
        C p2 = C{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
        C q2 = C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
        v[0] = C{x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
        v[1] = C{p1.x + q1.y, p1.y - q1.x};
        v[4] = C{p1.x - q1.y, p1.y + q1.x};
        v[2] = C{p2.x + q2.y, p2.y - q2.x};
        v[3] = C{p2.x - q2.y, p2.y + q2.x};
    }
}

// In-place forward DFT of N values (2,3,5-smooth), natural order in and out:
// N = P Q, n = Q n_p + n_q, k = k_p + P k_q.
template <typename T, int N>
__device__ __forceinline__ void dft_reg(typename CTf<T>::type* x)
{
    using C = typename CTf<T>::type;
    if constexpr (N <= 1) {
        return;
    } else if constexpr (N <= 5) {
        dft_small<T, N>(x);
    } else {
        constexpr int P = (N % 4 == 0 && N != 8) ? 4 : (N % 5 == 0 ? 5 : (N % 3 == 0 ? 3 : (N % 4 == 0 ? 4 : 2)));
        constexpr int Q = N / P;
        C t[N];
#pragma unroll
        for (int nq = 0; nq < Q; ++nq) {
            C v[P];
#pragma unroll
            for (int np = 0; np < P; ++np) v[np] = x[Q * np + nq];
            dft_small<T, P>(v);
#pragma unroll
            for (int kp = 0; kp < P; ++kp) t[nq * P + kp] = twc<T, N>(v[kp], nq * kp);
        }
#pragma unroll
        for (int kp = 0; kp < P; ++kp) {
            C u[Q];
#pragma unroll
            for (int nq = 0; nq < Q; ++nq) u[nq] = t[nq * P + kp];
            dft_reg<T, Q>(u);
#pragma unroll
            for (int kq = 0; kq < Q; ++kq) x[kp + P * kq] = u[kq];
        }
    }
}

template <typename C>
__device__ __forceinline__ C cmulf(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// W^m from the split table: lo[m & (LO-1)] * hi[m >> lo_bits].
template <typename C>
__device__ __forceinline__ C tw_split(const C* lo, const C* hi, int m, int lo_bits)
{
    return cmulf(lo[m & ((1 << lo_bits) - 1)], hi[m >> lo_bits]);
}

// ---------------------------------------------------------------- column pass
// Step A of one column: values n = B n_a + nb (n_a < A) straight from the grid,
// size-A DFT, times W_L1^{nb k_a}, into LDS block k_a.
template <typename T, int A>
__device__ __forceinline__ void col_step_a(const typename CTf<T>::type* z, int L2p, int B, int nb, int col,
                                           const typename CTf<T>::type* tw1, typename CTf<T>::type* sh, int blk,
                                           int slot)
{
    using C = typename CTf<T>::type;
    C x[A];
#pragma unroll
    for (int a = 0; a < A; ++a) x[a] = z[(int64_t)(B * a + nb) * L2p + col];
    dft_reg<T, A>(x);
#pragma unroll
    for (int a = 0; a < A; ++a) sh[a * blk + slot] = a ? cmulf(x[a], tw1[nb * a]) : x[a];
}

// Step B of one column: LDS block ka, size-B DFT, outputs k1 = ka + A k_b times
// the four-step twiddle W_L^{k1 col}, back to the grid.
template <typename T, int B>
__device__ __forceinline__ void col_step_b(typename CTf<T>::type* z, int L2p, int A, int ka, int col, int C_,
                                           const typename CTf<T>::type* sh, int blk, int c,
                                           const typename CTf<T>::type* lo, const typename CTf<T>::type* hi,
                                           int lo_bits)
{
    using C = typename CTf<T>::type;
    C y[B];
#pragma unroll
    for (int b = 0; b < B; ++b) y[b] = sh[ka * blk + b * C_ + c];
    dft_reg<T, B>(y);
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int k1 = ka + A * b;
        z[(int64_t)k1 * L2p + col] = cmulf(y[b], tw_split(lo, hi, k1 * col, lo_bits));
    }
}

#define MM_CODELETS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(9) X(10) X(12) X(15) X(16) X(18) X(20) X(24) \
    X(25) X(27) X(30) X(32)

// ---------------------------------------------------------------- row pass
template <typename T, int A>
__device__ __forceinline__ void row_step_a(const typename CTf<T>::type* row, int B, int nb,
                                           const typename CTf<T>::type* tw2, typename CTf<T>::type* shrow)
{
    using C = typename CTf<T>::type;
    C x[A];
#pragma unroll
    for (int a = 0; a < A; ++a) x[a] = row[B * a + nb];
    dft_reg<T, A>(x);
#pragma unroll
    for (int a = 0; a < A; ++a) shrow[a * B + nb] = a ? cmulf(x[a], tw2[nb * a]) : x[a];
}

// Step B of one row: reads block ka of the row into registers; after the barrier
// the caller stores the outputs (natural positions ka + A k_b) from y.
template <typename T, int B>
__device__ __forceinline__ void row_step_b(const typename CTf<T>::type* shrow, int ka, typename CTf<T>::type* y)
{
#pragma unroll
    for (int b = 0; b < B; ++b) y[b] = shrow[ka * B + b];
    dft_reg<T, B>(y);
}

template <typename T, int B>
__device__ __forceinline__ void row_store_b(typename CTf<T>::type* shrow, int A, int ka,
                                            const typename CTf<T>::type* y)
{
#pragma unroll
    for (int b = 0; b < B; ++b) shrow[ka + A * b] = y[b];
}

}  // namespace mm
