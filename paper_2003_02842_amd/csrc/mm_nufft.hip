// gfx950 kernels of the type-1 NUFFT (Sec. 2.2.5 of the paper):
//   k_prep         FP64 tables of the generic FFT passes: twiddles, digit-reversal maps
//   k_deconv       deconvolution factors 1/(2 pi psi_hat(k/Mr)) of the averaging
//                  kernel, one wave per k
//   k_tile_ranges  per (series, grid tile) event ranges by binary search on the
//                  sorted event keys
//   k_setup        with the two-pass FFT: the deconvolution factors, its twiddle
//                  tables and the tile ranges in one launch
//   k_spread       spreading onto the periodic oversampled grid (Eq. Der:15), one
//                  workgroup per (series, grid tile), each cell gathering its
//                  events from LDS and evaluating the kernel formula per pair; no
//                  atomics
//   k_spread_poly  the same sum in FP32 from per-tap polynomials evaluated once per
//                  event into LDS rings, then gathered per cell pair
//   k_fft_cols, k_fft_rows
//                  generic grid FFT (Eq. Der:16) with in-LDS mixed-radix passes,
//                  used where the two-pass register-codelet form (mm_fft.hip)
//                  does not apply: length-L1 transforms of the strided columns of
//                  the L1 x L2 view of the packed complex grid times the four-step
//                  twiddle, then length-L2 transforms of the rows with the
//                  real-input untangling, deconvolution (Eq. Der:17) and the 1/2pi
//                  of the coefficient definition; writes c_k, k = 0..N
//
// The real grid x[0..Mr) is FFT'd as the complex sequence z_j = x_2j + i x_2j+1
// of length L = Mr/2 = L1 L2; in the generic passes every sub-transform is an
// in-place mixed-radix (4, 5, 3, 2) decimation-in-frequency FFT in LDS whose
// output sits in digit-reversed positions.
#include <hip/hip_runtime.h>

#include "mm_fft_codelets.h"
#include "mm_internal.h"
#include "mm_spread.h"

// Events staged per LDS chunk by the per-pair FP32 spreading kernel (a multiple of 256).
#ifndef MM_SPREAD_CHUNK
#define MM_SPREAD_CHUNK 2048
#endif

namespace mm {

template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };

__device__ __forceinline__ uint32_t fdiv(uint32_t a, const FastDiv& f)
{
    return (uint32_t)(((uint64_t)a * f.M) >> 42);
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }
// -i * a
template <typename C> __device__ __forceinline__ C cmi(C a) { return C{a.y, -a.x}; }
// +i * a
template <typename C> __device__ __forceinline__ C cpi(C a) { return C{-a.y, a.x}; }

// In-place forward DFT of R values (R = 2, 3, 4, 5), exp(-2 pi i/R).
template <typename T, int R>
__device__ __forceinline__ void dft(typename CT<T>::type* v)
{
    using C = typename CT<T>::type;
    if constexpr (R == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T s3 = (T)0.86602540378443864676;
        C t1 = cadd(v[1], v[2]);
        C t2 = C{v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
        C t3 = cscale(csub(v[1], v[2]), s3);
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, cmi(t3));
        v[2] = cadd(t2, cpi(t3));
    } else if constexpr (R == 4) {
        C a = cadd(v[0], v[2]), b = csub(v[0], v[2]), c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, cmi(d));
        v[3] = cadd(b, cpi(d));
    } else {
        const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
        C x0 = v[0];
        C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]), a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        C p1 = C{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
        C q1 = C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
        C p2 = C{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
        C q2 = C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
        v[0] = cadd(x0, cadd(a1, a2));
        v[1] = cadd(p1, cmi(q1));
        v[4] = cadd(p1, cpi(q1));
        v[2] = cadd(p2, cmi(q2));
        v[3] = cadd(p2, cpi(q2));
    }
}

// One task of an LDS pass: the R1*R2 values base[q1 m1 + q2 m2] go through
// DIF stage A (radix R1, span len = R1 m1, butterfly index j = j2 + q2 m2,
// output q1' times W_len^{j q1'}) and, if R2 > 1, stage B on each of the R1
// sub-blocks (radix R2, span m1, butterfly index j2, output q2' times
// W_m1^{j2 q2'}), all in registers.  tw[i] = W_n^i, ts1 = n/len, ts2 = n/m1.
template <typename T, int R1, int R2>
__device__ __forceinline__ void pass_task(typename CT<T>::type* base, int m1, int m2, int j2, int ts1, int ts2,
                                          const typename CT<T>::type* tw)
{
    using C = typename CT<T>::type;
    C x[R1][R2];
#pragma unroll
    for (int a = 0; a < R1; ++a)
#pragma unroll
        for (int b = 0; b < R2; ++b) x[a][b] = base[a * m1 + b * m2];
#pragma unroll
    for (int b = 0; b < R2; ++b) {
        C v[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) v[a] = x[a][b];
        dft<T, R1>(v);
        const int j = j2 + b * m2;
        if (j) {
#pragma unroll
            for (int a = 1; a < R1; ++a) v[a] = cmul(v[a], tw[j * a * ts1]);
        }
#pragma unroll
        for (int a = 0; a < R1; ++a) x[a][b] = v[a];
    }
    if constexpr (R2 > 1) {
#pragma unroll
        for (int a = 0; a < R1; ++a) {
            C v[R2];
#pragma unroll
            for (int b = 0; b < R2; ++b) v[b] = x[a][b];
            dft<T, R2>(v);
            if (j2) {
#pragma unroll
                for (int b = 1; b < R2; ++b) v[b] = cmul(v[b], tw[j2 * b * ts2]);
            }
#pragma unroll
            for (int b = 0; b < R2; ++b) x[a][b] = v[b];
        }
    }
#pragma unroll
    for (int a = 0; a < R1; ++a)
#pragma unroll
        for (int b = 0; b < R2; ++b) base[a * m1 + b * m2] = x[a][b];
}

template <typename T, int R1>
__device__ __forceinline__ void pass_task_r2(int r2, typename CT<T>::type* base, int m1, int m2, int j2, int ts1,
                                             int ts2, const typename CT<T>::type* tw)
{
    switch (r2) {
        case 1: pass_task<T, R1, 1>(base, m1, m2, j2, ts1, ts2, tw); break;
        case 2: pass_task<T, R1, 2>(base, m1, m2, j2, ts1, ts2, tw); break;
        case 3: pass_task<T, R1, 3>(base, m1, m2, j2, ts1, ts2, tw); break;
        case 4: pass_task<T, R1, 4>(base, m1, m2, j2, ts1, ts2, tw); break;
        default: pass_task<T, R1, 5>(base, m1, m2, j2, ts1, ts2, tw); break;
    }
}

// nb independent length-n transforms, transform b at buf + b*ldb (unit stride),
// in place by decimation in frequency; the output sits in digit-reversed order.
// tw holds W_n^j = exp(-2 pi i j/n), j < n.  Ends with a barrier.
template <typename T>
__device__ void fft_lds(typename CT<T>::type* buf, int ldb, int nb, const FFTDesc& F,
                        const typename CT<T>::type* tw)
{
    for (int q = 0; q < F.np; ++q) {
        const int r1 = F.p1[q], r2 = F.p2[q], m1 = F.pm1[q], m2 = F.pm2[q], len = F.plen[q];
        const int ts1 = F.pts1[q], ts2 = F.pts2[q];
        const int tasks = (int)F.pdtask[q].d;
        const int total = nb * tasks;
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int b = (int)fdiv((uint32_t)idx, F.pdtask[q]);
            const int tsk = idx - b * tasks;
            const int blk = (int)fdiv((uint32_t)tsk, F.pdm2[q]);
            const int j2 = tsk - blk * m2;
            typename CT<T>::type* base = buf + b * ldb + blk * len + j2;
            switch (r1) {
                case 2: pass_task_r2<T, 2>(r2, base, m1, m2, j2, ts1, ts2, tw); break;
                case 3: pass_task_r2<T, 3>(r2, base, m1, m2, j2, ts1, ts2, tw); break;
                case 4: pass_task_r2<T, 4>(r2, base, m1, m2, j2, ts1, ts2, tw); break;
                default: pass_task_r2<T, 5>(r2, base, m1, m2, j2, ts1, ts2, tw); break;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// Time -> grid reduction (FP64).  u = (t - t0)/(T - t0), g = u Mr; first tap
// l0 = floor(g - hw) + 1 and fraction f = frac(g - hw), so tap j sits at cell
// l0 + j at kernel argument x_j = j + 1 - f - hw in (-hw, hw].  The key l0 is
// nondecreasing in t, which the per-tile binary searches rely on.  On the FP64
// path g is formed exactly as p + e (two-product).
//
// The mixed path (EXACT = false) needs the cell position only to ~1e-9 cells (it
// becomes an FP32 offset), so it forms g = (t - t0) (Mr/(T - t0)) with ordinary
// FP64 rounding; the FP64 path divides exactly like the definition and keeps the
// error-free product.  Either form is monotone in t.
template <bool EXACT>
__device__ __forceinline__ void cell_of(double t, double t0, double span, double scale, int Mr, double hw,
                                        int64_t& l0, double& f)
{
    // Explicitly rounded operations: the tile-range search and the spreading must
    // compute bit-identical keys, so no contraction may differ between them.
    if (EXACT) {
        double u = __ddiv_rn(__dsub_rn(t, t0), span);
        double p = __dmul_rn(u, (double)Mr);
        double e = fma(u, (double)Mr, -p);
        double tt = __dsub_rn(p, hw);
        double fl = floor(tt);
        double fr = __dadd_rn(__dsub_rn(tt, fl), e);
        if (fr < 0.0) { fl -= 1.0; fr += 1.0; }
        if (fr >= 1.0) { fl += 1.0; fr -= 1.0; }
        l0 = (int64_t)fl + 1;
        f = fr;
    } else {
        double tt = fma(__dsub_rn(t, t0), scale, -hw);
        double fl = floor(tt);
        l0 = (int64_t)fl + 1;
        f = __dsub_rn(tt, fl);
    }
}

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Kernel constants in the working precision, prepared once per thread.
template <typename T>
struct KEval {
    T inv_hw, es_c;        // ES: exp(beta (sqrt(1 - (x/hw)^2) - 1)); es_c = beta (log2 e for FP32)
    T g_c;                 // Gaussian: exp(-t1 x^2); g_c = t1 (times log2 e for FP32)
    T g_off;               // Gaussian: 1 - hw, so that x = (j + g_off) - f
    T kb_m2, kb_b, kb_inv_norm;
    __device__ explicit KEval(const KernParams& kp)
    {
        const double l2e = (sizeof(T) == 4) ? 1.4426950408889634074 : 1.0;
        inv_hw = (T)kp.es_inv_hw;
        es_c = (T)(kp.es_beta * l2e);
        g_c = (T)(kp.g_t1 * l2e);
        g_off = (T)(1.0 - kp.hw);
        kb_m2 = (T)(kp.kb_m * kp.kb_m);
        kb_b = (T)kp.kb_b;
        kb_inv_norm = (T)kp.kb_inv_norm;
    }
};

// The averaging kernel at cell distance x (|x| <= w/2), normalised to 1 at 0:
//   ES  exp(beta (sqrt(1 - (x/hw)^2) - 1))          (Eq. Der:10, support w cells)
//   G   exp(-t1 x^2), t1 = pi / lambda               (Eq. Der:5 in cells)
//   KB  inv_norm sinh(b s)/s, s = sqrt(m^2 - x^2),   (Eq. Der:8 in cells; sin(b s')/s'
//       s' = sqrt(x^2 - m^2) beyond |x| = m)
template <typename T, int KIND>
__device__ __forceinline__ T kern_eval(T x, const KEval<T>& k)
{
    if (KIND == MM_ES) {
        T z = x * k.inv_hw;
        if constexpr (sizeof(T) == 4) return fexp2(k.es_c * (fsqrt(fmaxf(1.0f - z * z, 0.0f)) - 1.0f));
        else return exp(k.es_c * (sqrt(fmax(1.0 - z * z, 0.0)) - 1.0));
    } else if (KIND == MM_GAUSSIAN) {
        if constexpr (sizeof(T) == 4) return fexp2(-k.g_c * x * x);
        else return exp(-k.g_c * x * x);
    } else {
        T s2 = k.kb_m2 - x * x;
        T val;
        if (s2 > (T)0) {
            T s = sqrt(s2);
            T a = k.kb_b * s;
            if constexpr (sizeof(T) == 4) {
                if (a < 0.5f) {
                    float a2 = a * a;
                    val = k.kb_b * (1.0f + a2 * (1.0f / 6 + a2 * (1.0f / 120 + a2 * (1.0f / 5040))));
                } else {
                    float E = expf(a);
                    val = (E - 1.0f / E) / (2.0f * s);
                }
            } else {
                val = sinh(a) / s;
            }
        } else if (s2 < (T)0) {
            T s = sqrt(-s2);
            val = sin(k.kb_b * s) / s;
        } else {
            val = k.kb_b;
        }
        return val * k.kb_inv_norm;
    }
}

// Event ranges of every (series, tile): for m = -1, 0, 1 the events whose taps
// [l0, l0 + w) meet cells [a, a + len) + m Mr, i.e. keys l0 in
// [a + m Mr - w + 1, a + len + m Mr); entry 2(m+1) is the first such event and
// 2(m+1)+1 one past the last (lower bounds on the sorted keys).
struct RangeJob {
    const int64_t* offsets;
    const double* t;
    int s_begin, s_count, tiles, tc, Mr, w;
    double hw, t0, span, scale;
    int64_t* ranges;
};

template <bool EXACT_DIV>
__device__ __forceinline__ void tile_range_at(const RangeJob& j, int64_t idx)
{
    const int64_t* __restrict__ offsets = j.offsets;
    const double* __restrict__ t = j.t;
    const int s_begin = j.s_begin, tiles = j.tiles, tc = j.tc, Mr = j.Mr, w = j.w;
    const double hw = j.hw, t0 = j.t0, span = j.span, scale = j.scale;
    const int q = (int)(idx % 6);
    const int64_t rest = idx / 6;
    const int tile = (int)(rest % tiles);
    const int s = s_begin + (int)(rest / tiles);
    const int64_t a = (int64_t)tile * tc;
    const int64_t len = min((int64_t)tc, (int64_t)Mr - a);
    const int64_t m = (int64_t)(q >> 1) - 1;
    const int64_t key = (q & 1) ? a + len + m * Mr : a + m * Mr - w + 1;
    int64_t lo = offsets[s], hi = offsets[s + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        int64_t l0;
        double f;
        cell_of<EXACT_DIV>(t[mid], t0, span, scale, Mr, hw, l0, f);
        if (l0 < key) lo = mid + 1;
        else hi = mid;
    }
    j.ranges[idx] = lo;
}

template <bool EXACT_DIV>
__global__ void k_tile_ranges(RangeJob j)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)j.s_count * j.tiles * 6) return;
    tile_range_at<EXACT_DIV>(j, idx);
}

// The three event ranges (m = -1, 0, 1) of spreading tile x of series s from the
// ranges of its sub-tiles of kRangeCells cells (nsub per series, rsub per tile):
// events are sorted by key, so range m runs from its first sub-tile's start to
// its last sub-tile's end.
__device__ __forceinline__ void tile_event_ranges(const int64_t* __restrict__ ranges, int s, int x, int nsub, int rsub,
                                                  int64_t (&rb)[3], int64_t (&re)[3])
{
    const int64_t* r0 = ranges + ((int64_t)s * nsub + (int64_t)x * rsub) * 6;
    const int64_t* r1 = ranges + ((int64_t)s * nsub + min(x * rsub + rsub, nsub) - 1) * 6;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        rb[m] = r0[2 * m];
        re[m] = r1[2 * m + 1];
    }
}

// One staged event.  key = first-tap cell relative to the tile plus w - 1 (a
// small integer held exactly as a float); the tap at cell c has index
// j = c + w - 1 - key and kernel argument x = j + x0 with x0 = 1 - f - hw.
// a is a per-event constant of the kernel in j:
//   ES  a = x0/hw           z = j/hw + a, value exp(beta (sqrt(1 - z^2) - 1))
//   G   a = f               x = (j + 1 - hw) - f, value exp(-t1 x^2) (FP32: exp2 with
//                           t1 log2 e); j + 1 - hw is exact, so x carries only the
//                           rounding of f, and the exponent is not formed by
//                           cancelling terms of size t1 x0^2
//   KB  a = x0              x = j + a
template <typename T>
struct EvRec {
    T key, a, v;
};
template <typename T, int KIND>
using EvRecK = EvRec<T>;

template <typename T, int KIND>
__device__ __forceinline__ EvRecK<T, KIND> make_rec(int key, double x0, T v, const KernParams& kp)
{
    EvRecK<T, KIND> r;
    r.key = (T)key;
    r.v = v;
    if constexpr (KIND == MM_ES) {
        r.a = (T)(x0 * kp.es_inv_hw);
    } else if constexpr (KIND == MM_GAUSSIAN) {
        r.a = (T)(1.0 - kp.hw - x0);
    } else {
        r.a = (T)x0;
    }
    return r;
}

// v * kernel at tap index j (as a float) of a staged event.
template <typename T, int KIND>
__device__ __forceinline__ T pair_value(T j, const EvRecK<T, KIND>& r, const KEval<T>& k)
{
    if (KIND == MM_ES) {
        const T z = fma(j, k.inv_hw, r.a);
        if constexpr (sizeof(T) == 4) {
            const float q = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
            return r.v * fexp2(fmaf(k.es_c, fsqrt(q), -k.es_c));
        } else {
            const double q = fmax(fma(-z, z, 1.0), 0.0);
            return r.v * exp(fma(k.es_c, sqrt(q), -k.es_c));
        }
    } else if (KIND == MM_GAUSSIAN) {
        const T x = (j + k.g_off) - r.a;
        if constexpr (sizeof(T) == 4) return r.v * fexp2(-k.g_c * x * x);
        else return r.v * exp(-k.g_c * x * x);
    } else {
        return r.v * kern_eval<T, MM_KAISER_BESSEL>(j + r.a, k);
    }
}

// Spreading (Eq. Der:15) by gathering: one workgroup per (series, tile of
// 256*CPT cells); thread tid owns cells tid + 256 r.  The tile's events, sorted
// by key, are staged in LDS in chunks together with first[k] = number of staged
// events with key < k; cell c then sums over the contiguous events with keys in
// [c, c + w - 1].  No atomics: each grid value is one thread's register sum.
template <typename T, typename DPT, int KIND, int CPT>
__global__ __launch_bounds__(256) void k_spread(const double* __restrict__ t, const DPT* __restrict__ dp,
                                                double t0, double span, double scale, KernParams kp, int Mr,
                                                const int64_t* __restrict__ ranges, int nsub, int rsub, int L2,
                                                int L2p, FastDiv divL2, T* __restrict__ grid, int64_t grid_stride)
{
    constexpr bool EXACT = sizeof(T) == 8;
    constexpr int TC = 256 * CPT;
    constexpr int EC = sizeof(T) == 4 ? MM_SPREAD_CHUNK : 1024;
    constexpr int SB = EC / 256;   // events per thread per chunk
    __shared__ EvRecK<T, KIND> ev[EC];
    __shared__ unsigned short first[TC + kMaxTaps + 2];
    const int a = blockIdx.x * TC;
    const int len = min(TC, Mr - a);
    const int w = kp.w;
    const KEval<T> ke(kp);
    // The three key ranges (m = -1, 0, 1) as one list of chunks of EC events.
    int64_t rb[3], re[3], nchunk[3];
    tile_event_ranges(ranges, blockIdx.y, blockIdx.x, nsub, rsub, rb, re);
    int total_chunks = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int64_t ne = re[m] - rb[m];
        nchunk[m] = (ne + EC - 1) / EC;
        total_chunks += (int)nchunk[m];
    }
    auto locate = [&](int q, int64_t& cb, int& n, int& m) {
        m = 0;
        while (q >= nchunk[m]) { q -= (int)nchunk[m]; ++m; }
        cb = rb[m] + (int64_t)q * EC;
        n = (int)min((int64_t)EC, re[m] - cb);
    };
    T acc[CPT];
#pragma unroll
    for (int r = 0; r < CPT; ++r) acc[r] = (T)0;
    double tv[SB];
    DPT dv[SB];
    if (total_chunks > 0) {
        int64_t cb; int n, m;
        locate(0, cb, n, m);
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int i = (int)threadIdx.x + 256 * u;
            if (i < n) { tv[u] = t[cb + i]; dv[u] = dp[cb + i]; }
        }
    }
    for (int q = 0; q < total_chunks; ++q) {
        int64_t cb; int n, m;
        locate(q, cb, n, m);
        const int64_t shift = (int64_t)a + (int64_t)(m - 1) * Mr;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int i = (int)threadIdx.x + 256 * u;
            if (i < n) {
                int64_t l0;
                double f;
                cell_of<EXACT>(tv[u], t0, span, scale, Mr, kp.hw, l0, f);
                ev[i] = make_rec<T, KIND>((int)(l0 - shift) + w - 1, 1.0 - f - kp.hw, (T)dv[u], kp);
            }
        }
        // prefetch the next chunk while this one is summed
        if (q + 1 < total_chunks) {
            int64_t cb2; int n2, m2;
            locate(q + 1, cb2, n2, m2);
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int i = (int)threadIdx.x + 256 * u;
                if (i < n2) { tv[u] = t[cb2 + i]; dv[u] = dp[cb2 + i]; }
            }
        }
        __syncthreads();
        const int kmin = (int)ev[0].key, kmax = (int)ev[n - 1].key;
        for (int i = 1 + threadIdx.x; i < n; i += 256) {
            const int k1 = (int)ev[i].key;
            for (int k = (int)ev[i - 1].key + 1; k <= k1; ++k) first[k] = (unsigned short)i;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < CPT; ++r) {
            const int c = threadIdx.x + 256 * r;
            if (c >= len || c + w - 1 < kmin || c > kmax) continue;
            const int lo = (c <= kmin) ? 0 : first[c];
            const int hi = (c + w > kmax) ? n : first[c + w];
            const T cw = (T)(c + w - 1);
            T s0 = (T)0, s1 = (T)0;
            int e = lo;
            for (; e + 1 < hi; e += 2) {
                const EvRecK<T, KIND> p0 = ev[e], p1 = ev[e + 1];
                s0 += pair_value<T, KIND>(cw - p0.key, p0, ke);
                s1 += pair_value<T, KIND>(cw - p1.key, p1, ke);
            }
            if (e < hi) {
                const EvRecK<T, KIND> p0 = ev[e];
                s0 += pair_value<T, KIND>(cw - p0.key, p0, ke);
            }
            acc[r] += s0 + s1;
        }
    }
    // real cell a + c is part (a + c) & 1 of complex entry j = (a + c) >> 1, which the
    // L1 x L2 view stores at row j / L2, column j % L2, rows L2p apart
    T* out = grid + (int64_t)blockIdx.y * grid_stride;
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        const int c = threadIdx.x + 256 * r;
        if (c < len) {
            const int cell = a + c, j = cell >> 1;
            const int row = (int)fdiv((uint32_t)j, divL2);
            out[2 * ((int64_t)row * L2p + (j - row * L2)) + (cell & 1)] = acc[r];
        }
    }
}

// FP32 spreading (Eq. Der:15) from per-tap polynomials, in two phases per chunk
// of staged events:
//   1. each thread evaluates all W taps of its events (tap j is a polynomial in
//      s = f - 1/2 whose coefficients are kernel arguments, so every lane runs the
//      same Horner chains on scalar operands) times the return.  Event i owns a
//      ring of M >= W+1 LDS slots; the tap for cell k goes to slot k mod M and the
//      M - W slots no tap reaches hold 0;
//   2. each thread gathers for its cell pairs (c, c+1), c even: the events with
//      keys c .. c+W (contiguous, sorted) reach cell c at slot c mod M and cell
//      c+1 at the next slot (M even, so the pair is one aligned 8-byte read), and an
//      event that reaches only one of the two cells reads a zero slot for the other.
// No load depends on another, so the gather streams LDS reads.  Cell pairs are the
// real and imaginary parts of one complex grid entry: one float2 store per pair.
// (spread_tile_poly in mm_spread.h is the same algorithm for the fused kernel; this
// kernel keeps its own copy, with its LDS arrays declared here, because as an inlined
// call the compiler allocates it 117 VGPRs instead of 78, which costs occupancy.)
template <typename DPT, int W, int PPT, int DEG>
__global__ __launch_bounds__(256) void k_spread_poly(const double* __restrict__ t, const DPT* __restrict__ dp,
                                                     double t0, double scale, int Mr, double hw, PolyParams pp,
                                                     const int64_t* __restrict__ ranges, int nsub, int rsub,
                                                     float dmin, int L2, int L2p, FastDiv divL2,
                                                     float* __restrict__ grid, int64_t grid_stride)
{
    constexpr int TC = 512 * PPT;
    constexpr int M = (W + 2) & ~1;                      // even ring, >= W + 1
    constexpr int EC = SpreadLds<W, PPT>::EC;                  // ~25 KB of LDS
    constexpr int SB = EC / 256;
    static_assert(DEG >= 4 && DEG <= kMaxPolyDeg, "polynomial degree");
    __shared__ __align__(8) float ring[EC * M];
    __shared__ unsigned short keys[EC];
    __shared__ unsigned short first[TC + W + 2];
    const int a = blockIdx.x * TC;
    const int len = min(TC, Mr - a);
    int64_t rb[3], re[3], nchunk[3];
    tile_event_ranges(ranges, blockIdx.y, blockIdx.x, nsub, rsub, rb, re);
    int total_chunks = 0;
    int64_t n_tile = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int64_t ne = re[m] - rb[m];
        n_tile += ne;
        nchunk[m] = (ne + EC - 1) / EC;
        total_chunks += (int)nchunk[m];
    }
    if ((float)n_tile >= dmin * (float)len) return;   // a dense tile: k_spread_mom's
    auto locate = [&](int q, int64_t& cb, int& n, int& m) {
        m = 0;
        while (q >= nchunk[m]) { q -= (int)nchunk[m]; ++m; }
        cb = rb[m] + (int64_t)q * EC;
        n = (int)min((int64_t)EC, re[m] - cb);
    };
    float acc0[PPT], acc1[PPT];
#pragma unroll
    for (int r = 0; r < PPT; ++r) acc0[r] = acc1[r] = 0.f;
    // leading coefficients of each tap's even and odd Horner chains, held in vector
    // registers for the whole kernel: the first step of a chain then reads one
    // scalar operand instead of two (one scalar operand per instruction)
    float ctop[(W + 1) / 2][2];
#pragma unroll
    for (int j = 0; j < (W + 1) / 2; ++j) {
        ctop[j][0] = pp.c[j][DEG & ~1];
        ctop[j][1] = pp.c[j][(DEG - 1) | 1];
        asm volatile("" : "+v"(ctop[j][0]), "+v"(ctop[j][1]));
    }
    // Chunk staging runs two chunks ahead: two register sets alternate, so that the
    // loads of chunk q+1 are already in flight while chunk q is staged, and those of
    // chunk q+2 are issued as soon as chunk q's registers are free.
    // The loads are unconditional (past the end of a chunk, or past the last chunk,
    // they repeat its last event), so every path issues the same loads and the
    // compiler's wait before staging a chunk leaves the other set in flight.
    auto load_chunk = [&](int qq, double (&tvx)[SB], DPT (&dvx)[SB]) {
        int64_t cb2; int n2, m2;
        locate(min(qq, total_chunks - 1), cb2, n2, m2);
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int64_t ii = cb2 + min((int)threadIdx.x + 256 * u, n2 - 1);
            tvx[u] = t[ii];
            dvx[u] = dp[ii];
        }
    };
    auto chunk = [&](int q, double (&tv)[SB], DPT (&dv)[SB]) {
        int64_t cb; int n, m;
        locate(q, cb, n, m);
        // key = first-tap cell - (a + (m - 1) Mr) + W - 1, the first-tap cell being floor(g - hw) + 1
        const int kofs = (int)((int64_t)W - (int64_t)a - (int64_t)(m - 1) * Mr);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int i = (int)threadIdx.x + 256 * u;
            if (i < n) {
                // cell_of<false> with the cell in 32 bits (|floor(g - hw)| < Mr + w < 2^31)
                const double tt = fma(__dsub_rn(tv[u], t0), scale, -hw);
                const double fl = floor(tt);
                const double f = __dsub_rn(tt, fl);
                const int key = (int)fl + kofs;              // >= 0; tap j reaches cell key - W + 1 + j
                const float sv = (float)(f - 0.5);
                const float v = (float)dv[u];
                // tap j = v (E_j(s^2) + s O_j(s^2)) and, by the kernel's symmetry, tap W-1-j =
                // v (E_j(s^2) - s O_j(s^2)): even and odd coefficients by Horner in s^2,
                // the return folded in as v E_j and (v s) O_j
                const float s2 = sv * sv, vs = v * sv;
                float tap[W];
#pragma unroll
                for (int j = 0; j < (W + 1) / 2; ++j) {
                    constexpr int DE = DEG & ~1, DO = (DEG - 1) | 1;   // top even and odd powers
                    float ev = fmaf(ctop[j][0], s2, pp.c[j][DE - 2]), od = fmaf(ctop[j][1], s2, pp.c[j][DO - 2]);
#pragma unroll
                    for (int k = DE - 4; k >= 0; k -= 2) ev = fmaf(ev, s2, pp.c[j][k]);
#pragma unroll
                    for (int k = DO - 4; k >= 1; k -= 2) od = fmaf(od, s2, pp.c[j][k]);
                    const float vev = v * ev;
                    tap[j] = fmaf(vs, od, vev);
                    if (W - 1 - j != j) tap[W - 1 - j] = fmaf(-vs, od, vev);
                }
                // slot of tap j: base + j, or base + j - M past the end of the ring; each
                // store picks one of two row pointers and adds j as a constant offset
                const int base = (key - W + 1 + M) % M;     // slot of tap 0: (key - W + 1) mod M, key >= 0
                const int r1 = 4 * (i * M + base), r2 = r1 - 4 * M;   // byte offsets of the two rows
                char* const rb = reinterpret_cast<char*>(ring);
#pragma unroll
                for (int j = 0; j < M; ++j)
                    *reinterpret_cast<float*>(rb + (j < M - base ? r1 : r2) + 4 * j) = j < W ? tap[j] : 0.f;
                keys[i] = (unsigned short)key;
            }
        }
        // this register set is free again: load the chunk after next into it
        load_chunk(q + 2, tv, dv);
        __syncthreads();
        // the chunk's key range, the same for every lane: held in scalar registers
        const int kmin = __builtin_amdgcn_readfirstlane(keys[0]);
        const int kmax = __builtin_amdgcn_readfirstlane(keys[n - 1]);
        for (int i = 1 + threadIdx.x; i < n; i += 256) {
            const int k1 = keys[i];
            for (int k = keys[i - 1] + 1; k <= k1; ++k) first[k] = (unsigned short)i;
        }
        __syncthreads();
        // rounds whose cell pairs (c, c+1), c = 2 (tid + 256 r), can meet the chunk:
        // kmin - W <= c <= kmax; the others are skipped by a scalar branch
        const int r_lo = max(kmin - W, 0) >> 9, r_hi = kmax >> 9;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            if (r < r_lo || r > r_hi) continue;
            const int c = 2 * ((int)threadIdx.x + 256 * r);
            if (c >= len || c + W < kmin || c > kmax) continue;
            const int lo = (c <= kmin) ? 0 : first[c];
            const int hi = (c + W + 1 > kmax) ? n : first[c + W + 1];
            const float2* rp = reinterpret_cast<const float2*>(ring + (c % M)) + (lo * M) / 2;
            float s0 = 0.f, s1 = 0.f, u0 = 0.f, u1 = 0.f, p0 = 0.f, p1 = 0.f, q0 = 0.f, q1 = 0.f;
            int e = lo;
            for (; e + 3 < hi; e += 4, rp += 2 * M) {
                const float2 x = rp[0], y = rp[M / 2], z = rp[M], zz = rp[3 * M / 2];
                s0 += x.x;
                s1 += x.y;
                u0 += y.x;
                u1 += y.y;
                p0 += z.x;
                p1 += z.y;
                q0 += zz.x;
                q1 += zz.y;
            }
            for (; e < hi; ++e, rp += M / 2) {
                const float2 x = rp[0];
                s0 += x.x;
                s1 += x.y;
            }
            acc0[r] += (s0 + u0) + (p0 + q0);
            acc1[r] += (s1 + u1) + (p1 + q1);
        }
        };
    double tva[SB], tvb[SB];
    DPT dva[SB], dvb[SB];
    if (total_chunks > 0) {
        load_chunk(0, tva, dva);
        load_chunk(1, tvb, dvb);
    }
    for (int q = 0; q < total_chunks; q += 2) {
        chunk(q, tva, dva);
        if (q + 1 >= total_chunks) break;
        chunk(q + 1, tvb, dvb);
    }
    // cells (c, c+1) are complex entry j = (a + c)/2 at row j / L2, column j % L2
    float2* out = reinterpret_cast<float2*>(grid + (int64_t)blockIdx.y * grid_stride);
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
        const int c = 2 * ((int)threadIdx.x + 256 * r);
        if (c < len) {
            const int j = (a + c) >> 1;
            const int row = (int)fdiv((uint32_t)j, divL2);
            out[(int64_t)row * L2p + (j - row * L2)] = make_float2(acc0[r], acc1[r]);
        }
    }
}

// Dense tiles: the same sum from per-cell moments.  Tap j of an event with offset
// s = f - 1/2 and return v is v p_j(s) = sum_d c_jd v s^d, so the events whose
// first tap is cell l give cell l + j the amount sum_d c_jd M_l[d], with the
// moments M_l[d] = sum over those events of v s^d, and
//   x_c = sum_{j < W} sum_{d <= DEG} c_jd M_{c-j}[d].
// Per event that is DEG multiplies and DEG+1 adds (no taps, no ring, no gather);
// per cell W (DEG+1) multiply-adds, so it pays once a tile holds more than about
// one event per cell.  This kernel takes the tiles with at least dmin events per
// cell and k_spread_poly the others (the same test in both).  A tile of tc cells
// runs as sub-tiles of kMomCells cells, each in three steps:
//   1. the sub-tile's event ranges (from the set-up's search, which is done per
//      sub-tile of kRangeCells cells);
//   2. per staged chunk ((s, v) in LDS, the first event of every key; the next
//      chunk's loads in flight meanwhile), thread t sums in registers the moments
//      of keys t, t + 256, t + 512, t + 768 over their events; the last W-1 keys
//      (past kMomCells) are summed into LDS by threads 0..W-2;
//   3. the moments go to LDS (over the staging buffers), and thread t forms cells
//      4t..4t+3 from keys 4t..4t+3+W-1.
// A key is the event's first-tap cell minus (b - W + 1), b the sub-tile's first
// cell: cell c of the sub-tile takes tap j from key c + W - 1 - j.  Every sum has
// a fixed order (events in time order per key, then d, then j), so results are
// reproducible bit for bit.
constexpr int kMomCells = 1024;   // cells of a sub-tile: 4 per thread
constexpr int kMomEV = 4;         // events per thread per staged chunk

template <int W, int DEG>
struct MomLds {
    static constexpr int ND = DEG + 1;                          // moments per key (<= 9)
    static constexpr int NKP = kMomCells + 16;                  // keys, padded (W <= 17)
    static constexpr int EC = kMomEV * 256;                     // events per chunk
    static constexpr int stage_bytes = 8 * EC + 2 * EC + 2 * (NKP + 2);
    static constexpr int mom_bytes = (ND > 8 ? 36 : 32) * NKP;  // per key: d 0-3, d 4-7 (float4), d 8
    static constexpr int bytes = stage_bytes > mom_bytes ? stage_bytes : mom_bytes;
};

template <typename DPT, int W, int DEG>
__global__ __launch_bounds__(256) void k_spread_mom(const double* __restrict__ t, const DPT* __restrict__ dp,
                                                    double t0, double scale, int Mr, double hw, PolyParams pp,
                                                    const int64_t* __restrict__ ranges, int nsub, int rsub, int tc,
                                                    float dmin, int L2, int L2p, FastDiv divL2,
                                                    float* __restrict__ grid, int64_t grid_stride)
{
    using Lay = MomLds<W, DEG>;
    constexpr int ND = Lay::ND, NKP = Lay::NKP, EC = Lay::EC;
    constexpr int H = (W + 1) / 2;                              // taps with stored coefficients
    static_assert(W >= 2 && W <= 17 && ND <= 9, "key padding, moment layout");
    __shared__ __align__(16) char lds[Lay::bytes];
    __shared__ float hmom[16 * ND];                             // keys kMomCells.. (their owners: threads 0..W-2)
    float2* const sv = reinterpret_cast<float2*>(lds);                              // staging: (s, v)
    unsigned short* const keys = reinterpret_cast<unsigned short*>(lds + 8 * EC);   // staging: keys
    unsigned short* const first = keys + EC;                                        // first event of a key
    float4* const momA = reinterpret_cast<float4*>(lds);                            // moments d 0-3
    float4* const momB = momA + NKP;                                                // d 4-7
    float* const momC = reinterpret_cast<float*>(momB + NKP);                       // d 8

    const int a = blockIdx.x * tc;
    const int len = min(tc, Mr - a);
    {
        int64_t tb[3], te[3], n_tile = 0;
        tile_event_ranges(ranges, blockIdx.y, blockIdx.x, nsub, rsub, tb, te);
#pragma unroll
        for (int m = 0; m < 3; ++m) n_tile += te[m] - tb[m];
        if (!((float)n_tile >= dmin * (float)len)) return;     // a sparse tile: k_spread_poly's
    }
    const int tid = threadIdx.x;
    float2* out = reinterpret_cast<float2*>(grid + (int64_t)blockIdx.y * grid_stride);

    static_assert(kMomCells == kRangeCells, "a sub-tile has its own event ranges");
    for (int b0 = 0, h = 0; b0 < len; b0 += kMomCells, ++h) {
        const int b = a + b0;
        const int lenh = min(kMomCells, len - b0);
        // 1. the sub-tile's event ranges (first-tap cells in [b + m' Mr - W + 1, b + lenh + m' Mr),
        //    m' = m - 1), from the set-up's search
        const int64_t* sr = ranges + ((int64_t)blockIdx.y * nsub + (int64_t)blockIdx.x * rsub + h) * 6;
        for (int i = tid; i < 16 * ND; i += 256) hmom[i] = 0.f;
        __syncthreads();
        int64_t rb[3], re[3], nchunk[3];
        int total_chunks = 0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            rb[m] = sr[2 * m];
            re[m] = max(sr[2 * m + 1], rb[m]);
            nchunk[m] = (re[m] - rb[m] + EC - 1) / EC;
            total_chunks += (int)nchunk[m];
        }
        auto locate = [&](int q, int64_t& cb, int& n, int& m) {
            m = 0;
            while (q >= nchunk[m]) { q -= (int)nchunk[m]; ++m; }
            cb = rb[m] + (int64_t)q * EC;
            n = (int)min((int64_t)EC, re[m] - cb);
        };
        // the chunk's loads are unconditional (past its end they repeat its last event)
        double tv[kMomEV];
        DPT dv[kMomEV];
        auto load_chunk = [&](int q) {
            int64_t cb; int n, m;
            locate(min(q, total_chunks - 1), cb, n, m);
#pragma unroll
            for (int u = 0; u < kMomEV; ++u) {
                const int64_t ii = cb + min(tid + 256 * u, n - 1);
                tv[u] = t[ii];
                dv[u] = dp[ii];
            }
        };
        float acc[4][ND];
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int d = 0; d < ND; ++d) acc[g][d] = 0.f;
        if (total_chunks > 0) load_chunk(0);

        // 2. chunks of staged events
        for (int q = 0; q < total_chunks; ++q) {
            int64_t cb; int n, m;
            locate(q, cb, n, m);
            // key = first-tap cell - (b + (m - 1) Mr) + W - 1, the first-tap cell being floor(g - hw) + 1
            const int kofs = (int)((int64_t)W - (int64_t)b - (int64_t)(m - 1) * Mr);
            __syncthreads();   // the previous chunk's staging is read out
#pragma unroll
            for (int u = 0; u < kMomEV; ++u) {
                const int i = tid + 256 * u;
                if (i < n) {
                    const double tt = fma(__dsub_rn(tv[u], t0), scale, -hw);
                    const double fl = floor(tt);
                    const double f = __dsub_rn(tt, fl);
                    sv[i] = make_float2((float)(f - 0.5), (float)dv[u]);
                    keys[i] = (unsigned short)((int)fl + kofs);
                }
            }
            if (q + 1 < total_chunks) load_chunk(q + 1);   // in flight while this chunk is summed
            __syncthreads();
            const int kmin = __builtin_amdgcn_readfirstlane(keys[0]);
            const int kmax = __builtin_amdgcn_readfirstlane(keys[n - 1]);
            for (int i = 1 + tid; i < n; i += 256) {
                const int k1 = keys[i];
                for (int k = keys[i - 1] + 1; k <= k1; ++k) first[k] = (unsigned short)i;
            }
            __syncthreads();
            // events of key k: [k <= kmin ? 0 : first[k], k >= kmax ? n : first[k + 1]), summed
            // in time order; four events' (s, v) are read at once, so their LDS reads
            // overlap (the adds stay in event order)
            auto add_event = [&](float2 x, float (&ac)[ND]) {
                float pw = x.y;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    ac[d] += pw;
                    if (d + 1 < ND) pw *= x.x;
                }
            };
            auto sum_key = [&](int k, float (&ac)[ND]) {
                const int lo = (k <= kmin) ? 0 : first[k];
                const int hi = (k >= kmax) ? n : first[k + 1];
                int e = lo;
                for (; e + 3 < hi; e += 4) {
                    const float2 x0 = sv[e], x1 = sv[e + 1], x2 = sv[e + 2], x3 = sv[e + 3];
                    add_event(x0, ac);
                    add_event(x1, ac);
                    add_event(x2, ac);
                    add_event(x3, ac);
                }
                for (; e < hi; ++e) add_event(sv[e], ac);
            };
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int k = tid + 256 * g;
                if (k >= kmin && k <= kmax) sum_key(k, acc[g]);
            }
            if (tid < W - 1) {
                const int k = kMomCells + tid;
                if (k >= kmin && k <= kmax) {
                    float h[ND];
#pragma unroll
                    for (int d = 0; d < ND; ++d) h[d] = hmom[tid * ND + d];
                    sum_key(k, h);
#pragma unroll
                    for (int d = 0; d < ND; ++d) hmom[tid * ND + d] = h[d];
                }
            }
        }
        // 3. moments to LDS (over the staging buffers), then the cells
        __syncthreads();
        auto put = [&](int k, const float* mv) {
            float v[9];
#pragma unroll
            for (int d = 0; d < 9; ++d) v[d] = d < ND ? mv[d] : 0.f;
            momA[k] = make_float4(v[0], v[1], v[2], v[3]);
            momB[k] = make_float4(v[4], v[5], v[6], v[7]);
            if (ND > 8) momC[k] = v[8];
        };
#pragma unroll
        for (int g = 0; g < 4; ++g) put(tid + 256 * g, acc[g]);
        if (tid < 16) {
            float h[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) h[d] = tid < W - 1 ? hmom[tid * ND + d] : 0.f;
            put(kMomCells + tid, h);
        }
        __syncthreads();
        if (4 * tid < lenh) {
            float x[4] = {0.f, 0.f, 0.f, 0.f};
            // keys 4t + kk, kk = 0 .. W + 2, one at a time (a uniform loop: the
            // coefficients are scalar loads)
#pragma unroll 1
            for (int kk = 0; kk < W + 3; ++kk) {
                const int k = 4 * tid + kk;
                const float4 A = momA[k], B = momB[k];
                const float m8 = ND > 8 ? momC[k] : 0.f;
                const float mv[9] = {A.x, A.y, A.z, A.w, B.x, B.y, B.z, B.w, m8};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = r + W - 1 - kk;               // tap of key 4t + kk reaching cell 4t + r
                    if (j < 0 || j >= W) continue;
                    const bool mir = j >= H;                    // the mirror of stored tap W-1-j: (-1)^d
                    const int js = mir ? W - 1 - j : j;
#pragma unroll
                    for (int d = 0; d < ND; ++d) {
                        const float c = pp.c[js][d];
                        x[r] = fmaf((mir && (d & 1)) ? -c : c, mv[d], x[r]);
                    }
                }
            }
            // cells (4t, 4t+1) and (4t+2, 4t+3): complex entries (b + 4t)/2 and (b + 4t)/2 + 1
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (4 * tid + 2 * h < lenh) {
                    const int j = (b + 4 * tid) / 2 + h;
                    const int row = (int)fdiv((uint32_t)j, divL2);
                    out[(int64_t)row * L2p + (j - row * L2)] = make_float2(x[2 * h], x[2 * h + 1]);
                }
            }
        }
        __syncthreads();   // the moments are read out before the next sub-tile stages over them
    }
}

template <typename DPT, int W, int DEG>
static void spread_poly_wd(const Plan& p, dim3 g, const double* t, const DPT* dp, double t0, double scale,
                           const int64_t* ranges, int nsub, float* grid, int64_t gs, hipStream_t st)
{
    const int rsub = p.tile / kRangeCells;
    const FastDiv dv = make_fastdiv((uint32_t)p.L2);
    // tiles with at least dmin events per cell go to the moment kernel (none if it is off)
    const bool mom = p.mom_density > 0.0 && W <= 17;
    const float dmin = mom ? (float)p.mom_density : __builtin_huge_valf();
    prof_begin("k_spread_poly", st);
    if (p.tile <= 1024)
        hipLaunchKernelGGL((k_spread_poly<DPT, W, 2, DEG>), g, dim3(256), 0, st, t, dp, t0, scale, p.Mr, p.kp.hw,
                           p.pp, ranges, nsub, rsub, dmin, p.L2, p.L2p, dv, grid, gs);
    else if (p.tile <= 2048)
        hipLaunchKernelGGL((k_spread_poly<DPT, W, 4, DEG>), g, dim3(256), 0, st, t, dp, t0, scale, p.Mr, p.kp.hw,
                           p.pp, ranges, nsub, rsub, dmin, p.L2, p.L2p, dv, grid, gs);
    else
        hipLaunchKernelGGL((k_spread_poly<DPT, W, 8, DEG>), g, dim3(256), 0, st, t, dp, t0, scale, p.Mr, p.kp.hw,
                           p.pp, ranges, nsub, rsub, dmin, p.L2, p.L2p, dv, grid, gs);
    prof_end("k_spread_poly", st);
    if (mom) {
        prof_begin("k_spread_mom", st);
        hipLaunchKernelGGL((k_spread_mom<DPT, W, DEG>), g, dim3(256), 0, st, t, dp, t0, scale, p.Mr, p.kp.hw, p.pp,
                           ranges, nsub, rsub, p.tile, dmin, p.L2, p.L2p, dv, grid, gs);
        prof_end("k_spread_mom", st);
    }
}

// The plan's polynomial degree: the width's own (poly_degree_for_width), or one
// less where the planner found that enough (kPolyDegLow, widths of degree-8 plans).
template <typename DPT, int W>
static void spread_poly_w(const Plan& p, dim3 g, const double* t, const DPT* dp, double t0, double scale,
                          const int64_t* ranges, int nsub, float* grid, int64_t gs, hipStream_t st)
{
    constexpr int D0 = poly_degree_for_width(W);
    if constexpr (D0 == kPolyDegTop) {
        if (p.pp.deg == kPolyDegLow) {
            spread_poly_wd<DPT, W, kPolyDegLow>(p, g, t, dp, t0, scale, ranges, nsub, grid, gs, st);
            return;
        }
    }
    spread_poly_wd<DPT, W, D0>(p, g, t, dp, t0, scale, ranges, nsub, grid, gs, st);
}

template <typename DPT>
static hipError_t spread_poly_t(const Plan& p, int s_count, const double* t, const DPT* dp, double t0, double t_end,
                                const int64_t* ranges, int nsub, float* grid, int64_t gs, hipStream_t st)
{
    const double span = t_end - t0;
    const double scale = (double)p.Mr / span;
    const dim3 g((p.Mr + p.tile - 1) / p.tile, s_count);
    switch (p.kp.w) {
#define MM_POLY_W(n) case n: spread_poly_w<DPT, n>(p, g, t, dp, t0, scale, ranges, nsub, grid, gs, st); break;
        MM_POLY_W(2) MM_POLY_W(3) MM_POLY_W(4) MM_POLY_W(5) MM_POLY_W(6) MM_POLY_W(7) MM_POLY_W(8) MM_POLY_W(9)
        MM_POLY_W(10) MM_POLY_W(11) MM_POLY_W(12) MM_POLY_W(13) MM_POLY_W(14) MM_POLY_W(15) MM_POLY_W(16)
#undef MM_POLY_W
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spread_poly(const Plan& p, int s_count, const double* t, const void* dp, int dp_fp64, double t0,
                              double t_end, const int64_t* ranges, int nsub, float* grid, int64_t grid_stride,
                              hipStream_t st)
{
    if (dp_fp64)
        return spread_poly_t<double>(p, s_count, t, (const double*)dp, t0, t_end, ranges, nsub, grid, grid_stride,
                                     st);
    return spread_poly_t<float>(p, s_count, t, (const float*)dp, t0, t_end, ranges, nsub, grid, grid_stride, st);
}

constexpr int kBatch = 8;   // independent global loads a thread issues before consuming them

// First FFT pass, in place on the packed complex grid viewed as an L1 x L2
// row-major matrix: workgroup (column block, series) transforms CB columns of
// length L1 and multiplies entry (k1, l2) by W_L^{k1 l2}.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_cols(T* __restrict__ grid, int64_t grid_stride, int L1, int L2, int L2p,
                                                  int cb_shift, FFTDesc F1, const typename CT<T>::type* __restrict__ tw1,
                                                  const typename CT<T>::type* __restrict__ twL,
                                                  const int* __restrict__ rev1)
{
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) char smem_raw[];
    C* tws = reinterpret_cast<C*>(smem_raw);
    int* rev = reinterpret_cast<int*>(tws + L1);
    C* buf = reinterpret_cast<C*>(rev + ((L1 + 3) & ~3));
    const int CB = 1 << cb_shift;
    const int ldb = L1 | 1;
    C* z = reinterpret_cast<C*>(grid + (int64_t)blockIdx.y * grid_stride);
    const int c0 = blockIdx.x * CB;
    const int nb = min(CB, L2 - c0);
    for (int i = threadIdx.x; i < L1; i += blockDim.x) {
        tws[i] = tw1[i];
        rev[i] = rev1[i];
    }
    const int total = L1 * CB;
    for (int base = 0; base < total; base += 256 * kBatch) {
        C v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            const int l1 = idx >> cb_shift, b = idx & (CB - 1);
            if (idx < total && b < nb) v[u] = z[(int64_t)l1 * L2p + c0 + b];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            const int l1 = idx >> cb_shift, b = idx & (CB - 1);
            if (idx < total && b < nb) buf[b * ldb + l1] = v[u];
        }
    }
    __syncthreads();
    fft_lds<T>(buf, ldb, nb, F1, tws);
    for (int base = 0; base < total; base += 256 * kBatch) {
        C tv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            const int p = idx >> cb_shift, b = idx & (CB - 1);
            if (idx < total && b < nb) tv[u] = twL[(int64_t)(c0 + b) * rev[p]];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            const int p = idx >> cb_shift, b = idx & (CB - 1);
            if (idx < total && b < nb) z[(int64_t)rev[p] * L2p + c0 + b] = cmul(buf[b * ldb + p], tv[u]);
        }
    }
}

// Second FFT pass: workgroup (row-pair block, series) loads rows k1 and
// L1 - k1 (mod L1) for R consecutive k1, transforms them (length L2), and writes
// c_k for k = k1 + L1 k2 <= N: the real-input untangling
//   X_k = (Z_k + conj Z_{L-k})/2 - (i/2) W_Mr^k (Z_k - conj Z_{L-k})
// (Z_{L-k} sits in the mirror row), then the deconvolution factor.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_rows(const T* __restrict__ grid, int64_t grid_stride, int L1, int L2, int L2p,
                                                  int r_shift, FFTDesc F2, FastDiv divL2,
                                                  const typename CT<T>::type* __restrict__ tw2,
                                                  const int* __restrict__ pos2, const typename CT<T>::type* __restrict__ twM,
                                                  const T* __restrict__ dfac, int N, typename CT<T>::type* __restrict__ coef,
                                                  int64_t ldc, int s_out)
{
    using C = typename CT<T>::type;
    extern __shared__ __align__(16) char smem_raw[];
    C* tws = reinterpret_cast<C*>(smem_raw);
    int* pos = reinterpret_cast<int*>(tws + L2);
    C* buf = reinterpret_cast<C*>(pos + ((L2 + 3) & ~3));
    const int R = 1 << r_shift;
    const int ldb = L2 | 1;
    const C* Y = reinterpret_cast<const C*>(grid + (int64_t)blockIdx.y * grid_stride);
    C* out = coef + (int64_t)(s_out + blockIdx.y) * ldc;
    const int P = L1 / 2 + 1;
    const int p0 = blockIdx.x * R;
    const int nr = min(R, P - p0);
    for (int i = threadIdx.x; i < L2; i += blockDim.x) {
        tws[i] = tw2[i];
        pos[i] = pos2[i];
    }
    // LDS row 2i holds matrix row p0+i, row 2i+1 its mirror (L1 - p0 - i) mod L1.
    const int total_in = 2 * nr * L2;
    for (int base = 0; base < total_in; base += 256 * kBatch) {
        C v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            if (idx < total_in) {
                const int row = (int)fdiv((uint32_t)idx, divL2), j = idx - row * L2;
                const int p = p0 + (row >> 1);
                const int k1 = (row & 1) ? (L1 - p) % L1 : p;
                v[u] = Y[(int64_t)k1 * L2p + j];
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            if (idx < total_in) {
                const int row = (int)fdiv((uint32_t)idx, divL2), j = idx - row * L2;
                buf[row * ldb + j] = v[u];
            }
        }
    }
    __syncthreads();
    fft_lds<T>(buf, ldb, 2 * nr, F2, tws);
    const int total = 2 * R * L2;
    for (int base = 0; base < total; base += 256 * kBatch) {
        C wk[kBatch];
        T dk[kBatch];
        int64_t kk[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * 256 + (int)threadIdx.x;
            const int i = idx & (R - 1);
            const int t2 = idx >> r_shift;
            const int side = t2 & 1, k2 = t2 >> 1;
            const int p = p0 + i;
            const int rowA = p, rowB = (L1 - p) % L1;
            const int k1 = side ? rowB : rowA;
            const int64_t k = (int64_t)k1 + (int64_t)L1 * k2;
            const bool ok = idx < total && i < nr && !(side && rowB == rowA) && k <= N;
            kk[u] = ok ? k : -1;
            if (ok) {
                wk[u] = twM[k];
                dk[u] = dfac[k];
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (kk[u] < 0) continue;
            const int idx = base + u * 256 + (int)threadIdx.x;
            const int i = idx & (R - 1);
            const int t2 = idx >> r_shift;
            const int side = t2 & 1, k2 = t2 >> 1;
            const int k1 = (int)(kk[u] - (int64_t)L1 * k2);
            const int k2m = (k1 == 0) ? (k2 == 0 ? 0 : L2 - k2) : (L2 - 1 - k2);
            const C Zk = buf[(2 * i + side) * ldb + pos[k2]];
            const C Zm = buf[(2 * i + 1 - side) * ldb + pos[k2m]];
            const C A = C{Zk.x + Zm.x, Zk.y - Zm.y};
            const C B = C{Zk.x - Zm.x, Zk.y + Zm.y};
            const C WB = cmul(wk[u], B);
            const T d = dk[u] * (T)0.5;
            out[kk[u]] = C{(A.x + WB.y) * d, (A.y - WB.x) * d};
        }
    }
}

struct GLRule {
    double x[kGLNodes], w[kGLNodes];
};

// Modified Bessel function I0 by its power series sum_j (x^2/4)^j / (j!)^2.
__device__ double bessel_i0(double x)
{
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int j = 1; j < 1000; ++j) {
        term *= q / ((double)j * (double)j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// 1/(2 pi psi_hat(nu)) at nu = k/Mr for the kernel in grid units.
__device__ double deconv_factor(const KernParams& kp, int k, int Mr, const GLRule& gl)
{
    const double pi = 3.14159265358979323846;
    const double nu = (double)k / (double)Mr;
    double ph;
    if (kp.kind == MM_GAUSSIAN) {
        ph = sqrt(kp.g_lambda) * exp(-pi * kp.g_lambda * nu * nu);
    } else if (kp.kind == MM_KAISER_BESSEL) {
        double a = kp.kb_b * kp.kb_b - (2.0 * pi * nu) * (2.0 * pi * nu);
        ph = pi * kp.kb_inv_norm * bessel_i0(kp.kb_m * sqrt(fmax(a, 0.0)));   // Eq. Der:9 in cells
    } else {
        // hw int_{-1}^{1} exp(beta (sqrt(1 - z^2) - 1)) cos(2 pi nu hw z) dz by Gauss-Legendre (Eq. Der:11)
        double acc = 0.0;
        for (int q = 0; q < kGLNodes; ++q) {
            double z = gl.x[q];
            double phi = exp(kp.es_beta * (sqrt(1.0 - z * z) - 1.0));
            acc += gl.w[q] * phi * cospi(2.0 * nu * kp.hw * z);
        }
        ph = 2.0 * kp.hw * acc;
    }
    return 1.0 / (2.0 * pi * ph);
}

__device__ int digit_rev(int p, const FFTDesc& F)
{
    int k = 0, mult = 1, rem = p;
    for (int s = 0; s < F.ns; ++s) {
        int q = rem / F.m[s];
        rem -= q * F.m[s];
        k += q * mult;
        mult *= F.r[s];
    }
    return k;
}

__device__ int digit_pos(int k, const FFTDesc& F)
{
    int p = 0;
    for (int s = 0; s < F.ns; ++s) {
        int q = k % F.r[s];
        k /= F.r[s];
        p += q * F.m[s];
    }
    return p;
}

template <typename T>
__global__ void k_prep(int L1, int L2, int L, int Mr, FFTDesc F1, FFTDesc F2, typename CT<T>::type* tw1,
                       typename CT<T>::type* tw2, typename CT<T>::type* twL, typename CT<T>::type* twM, int* rev1,
                       int* pos2)
{
    using C = typename CT<T>::type;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto tw = [](int64_t j, int64_t n) {
        double s, c;
        sincospi(2.0 * (double)j / (double)n, &s, &c);
        return C{(T)c, (T)-s};
    };
    if (i < L1) { tw1[i] = tw(i, L1); return; }
    i -= L1;
    if (i < L2) { tw2[i] = tw(i, L2); return; }
    i -= L2;
    if (i < L) { twL[i] = tw(i, L); return; }
    i -= L;
    if (i < L) { twM[i] = tw(i, Mr); return; }
    i -= L;
    if (i < L1) { rev1[i] = digit_rev((int)i, F1); return; }
    i -= L1;
    if (i < L2) { pos2[i] = digit_pos((int)i, F2); return; }
}

// Deconvolution factors 1/(2 pi psi_hat(k/Mr)), k = 0..N: one wave per k.  The ES
// transform (Eq. Der:11) is a Gauss-Legendre sum over the rule's 2 x 64 symmetric
// nodes, one node per lane, added up by lane shuffles; the Gaussian and KB
// transforms have closed forms (lane 0).
// Column factors of the split fused into the row pass (SplitOut): for column
// c = (k mod L1) K2 + k / L1, c < ncol, the factor s_k d_k / 2, or 0 where k > N.
struct FacJob {
    const float* scale;   // s_k
    float* fac;           // nullptr: no fused split
    int L1, k2n, ncol;
};

template <typename T>
__device__ __forceinline__ void deconv_wave(int k, int q, int N, int Mr, const KernParams& kp, const GLRule& gl,
                                            T* __restrict__ dfac, const FacJob& fj)
{
    if (k > N) {
        if (q == 0 && fj.fac && k < fj.ncol) fj.fac[(k % fj.L1) * fj.k2n + k / fj.L1] = 0.f;
        return;
    }
    const double pi = 3.14159265358979323846;
    double d;
    if (kp.kind == MM_ES) {
        const double nu = (double)k / (double)Mr;
        double acc = 0.0;
        for (int n = q; n < kGLNodes; n += 64) {
            const double z = gl.x[n];
            acc += gl.w[n] * exp(kp.es_beta * (sqrt(1.0 - z * z) - 1.0)) * cospi(2.0 * nu * kp.hw * z);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
        d = 1.0 / (2.0 * pi * (2.0 * kp.hw * acc));
    } else {
        if (q != 0) return;
        d = deconv_factor(kp, k, Mr, gl);
    }
    if (q == 0) {
        dfac[k] = (T)d;
        if (fj.fac) fj.fac[(k % fj.L1) * fj.k2n + k / fj.L1] = (float)(0.5 * d * (double)fj.scale[k]);
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_deconv(int N, int Mr, KernParams kp, GLRule gl, T* __restrict__ dfac)
{
    deconv_wave<T>(blockIdx.x, threadIdx.x, N, Mr, kp, gl, dfac, FacJob{nullptr, nullptr, 1, 0, 0});
}

// The set-up of a two-pass-FFT plan in one launch of 256-thread blocks: blocks
// [0, nb_dec) the deconvolution factors (one wave per k, as k_deconv) and the
// fused split's column factors (fj), the next nb_tab blocks the FFT's twiddle
// tables (as k_fft_tables), the rest the tile event ranges of rj (as
// k_tile_ranges; none if rj.s_count is 0).
template <typename T, bool EXACT_DIV>
__global__ __launch_bounds__(256) void k_setup(int N, int Mr, KernParams kp, GLRule gl, T* __restrict__ dfac,
                                               FacJob fj, int nb_dec, FftTables<T> tb, int nb_tab, RangeJob rj)
{
    const int b = blockIdx.x;
    if (b < nb_dec) {
        deconv_wave<T>(4 * b + ((int)threadIdx.x >> 6), (int)threadIdx.x & 63, N, Mr, kp, gl, dfac, fj);
    } else if (b < nb_dec + nb_tab) {
        fft_tables_at<T>(tb, (int64_t)(b - nb_dec) * 256 + threadIdx.x);
    } else {
        const int64_t idx = (int64_t)(b - nb_dec - nb_tab) * 256 + threadIdx.x;
        if (idx < (int64_t)rj.s_count * rj.tiles * 6) tile_range_at<EXACT_DIV>(rj, idx);
    }
}

__global__ void k_validate(int32_t S, const int64_t* __restrict__ offsets, const double* __restrict__ t,
                           const void* __restrict__ dp, int dp_fp64, double t0, double T, int* flag)
{
    const int s = blockIdx.y;
    const int64_t e0 = offsets[s], e1 = offsets[s + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (s == 0 && e0 != 0) atomicOr(flag, 1);
        if (e1 < e0) atomicOr(flag, 1);
    }
    if (e1 < e0) return;
    int bad = 0;
    for (int64_t i = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < e1;
         i += (int64_t)gridDim.x * blockDim.x) {
        double ti = t[i];
        double di = dp_fp64 ? ((const double*)dp)[i] : (double)((const float*)dp)[i];
        if (!isfinite(ti) || !(ti >= t0) || !(ti <= T)) bad |= 2;
        if (!isfinite(di)) bad |= 4;
        if (i > e0 && !(t[i - 1] <= ti)) bad |= 8;
    }
    if (bad) atomicOr(flag, bad);
}

static GLRule host_gl()
{
    struct Rule {
        GLRule g;
        Rule() { gauss_legendre_pos(kGLNodes, g.x, g.w); }
    };
    static const Rule rule;   // built once, thread-safe (C++11 function-local static)
    return rule.g;
}

template <typename T>
static void setup_t(const Plan& p, const NufftWs& w, char* ws, const GLRule& gl, const RangeJob& rj,
                    int64_t n_ranges, const FacJob& fj, hipStream_t st)
{
    const int nk = fj.fac ? std::max(p.N + 1, fj.ncol) : p.N + 1;
    const int nb_dec = (nk + 3) / 4;
    const int nb_tab = (int)((fft_tables_count(p) + 255) / 256);
    const int nb_rng = (int)((n_ranges + 255) / 256);
    if (p.prec == MM_PLAIN_FP64)
        hipLaunchKernelGGL((k_setup<T, true>), dim3(nb_dec + nb_tab + nb_rng), dim3(256), 0, st, p.N, p.Mr, p.kp, gl,
                           (T*)(ws + w.dfac), fj, nb_dec, fft_tables_of<T>(p, w, ws), nb_tab, rj);
    else
        hipLaunchKernelGGL((k_setup<T, false>), dim3(nb_dec + nb_tab + nb_rng), dim3(256), 0, st, p.N, p.Mr, p.kp, gl,
                           (T*)(ws + w.dfac), fj, nb_dec, fft_tables_of<T>(p, w, ws), nb_tab, rj);
}

hipError_t launch_prep(const Plan& p, const NufftWs& w, char* ws, hipStream_t st, const RangeReq* rr,
                       const SplitOut* so)
{
    if (so && (!p.fft_ab || p.prec != MM_MIXED || so->k2n < 1 || (int64_t)p.L1 * so->k2n > so->kp2 ||
               (int64_t)p.L1 * so->k2n < (int64_t)p.N + 1 || so->k2n > p.L2))
        return hipErrorInvalidValue;   // the fused split runs only with the two-pass FFT, on its own layout
    const FacJob fj = so ? FacJob{so->scale, so->fac, p.L1, so->k2n, p.L1 * so->k2n} : FacJob{nullptr, nullptr, 1, 0, 0};
    GLRule gl = host_gl();
    if (p.fft_ab) {
        // deconvolution factors, twiddle tables and (if asked) tile ranges: one launch
        RangeJob rj{};
        int64_t nr = 0;
        if (rr && rr->s_count > 0) {
            const double span = rr->T - rr->t0;
            rj = RangeJob{rr->offsets, rr->t, rr->s_begin, rr->s_count, rr->tiles, rr->tc, p.Mr, p.kp.w, p.kp.hw,
                          rr->t0, span, (double)p.Mr / span, rr->ranges};
            nr = (int64_t)rr->s_count * rr->tiles * 6;
        }
        prof_begin("k_setup", st);
        if (p.prec == MM_MIXED) setup_t<float>(p, w, ws, gl, rj, nr, fj, st);
        else setup_t<double>(p, w, ws, gl, rj, nr, fj, st);
        prof_end("k_setup", st);
        return hipGetLastError();
    }
    // the generic FFT passes' tables
    const int64_t total = 2ll * p.L1 + 2ll * p.L2 + 2ll * p.L;
    const int blocks = (int)((total + 255) / 256);
    prof_begin("k_prep", st);
    if (p.prec == MM_MIXED)
        hipLaunchKernelGGL(k_prep<float>, dim3(blocks), dim3(256), 0, st, p.L1, p.L2, p.L, p.Mr, p.F1, p.F2,
                           (float2*)(ws + w.tw1), (float2*)(ws + w.tw2), (float2*)(ws + w.twL),
                           (float2*)(ws + w.twM), (int*)(ws + w.rev1), (int*)(ws + w.pos2));
    else
        hipLaunchKernelGGL(k_prep<double>, dim3(blocks), dim3(256), 0, st, p.L1, p.L2, p.L, p.Mr, p.F1, p.F2,
                           (double2*)(ws + w.tw1), (double2*)(ws + w.tw2), (double2*)(ws + w.twL),
                           (double2*)(ws + w.twM), (int*)(ws + w.rev1), (int*)(ws + w.pos2));
    prof_end("k_prep", st);
    prof_begin("k_deconv", st);
    if (p.prec == MM_MIXED)
        hipLaunchKernelGGL(k_deconv<float>, dim3(p.N + 1), dim3(64), 0, st, p.N, p.Mr, p.kp, gl,
                           (float*)(ws + w.dfac));
    else
        hipLaunchKernelGGL(k_deconv<double>, dim3(p.N + 1), dim3(64), 0, st, p.N, p.Mr, p.kp, gl,
                           (double*)(ws + w.dfac));
    prof_end("k_deconv", st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && rr)
        e = launch_tile_ranges(p, rr->offsets, rr->t, rr->s_begin, rr->s_count, rr->tiles, rr->tc, rr->t0, rr->T,
                               rr->ranges, st);
    return e;
}

hipError_t launch_validate(int32_t S, const int64_t* offsets, const double* t, const void* dp, int dp_fp64,
                           double t0, double T, int* flag, hipStream_t st)
{
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(64, S), dim3(256), 0, st, S, offsets, t, dp, dp_fp64, t0, T, flag);
    return hipGetLastError();
}

template <typename T, typename DPT, int KIND>
static void launch_spread_t(const Plan& p, int s_count, const double* t, const DPT* dp, double t0, double t_end,
                            const int64_t* ranges, int nsub, T* grid, int64_t grid_stride, hipStream_t st)
{
    const double span = t_end - t0;
    const double scale = (double)p.Mr / span;
    const dim3 g((p.Mr + p.tile - 1) / p.tile, s_count);
    const int rsub = p.tile / kRangeCells;
    if (p.tile <= 1024)
        hipLaunchKernelGGL((k_spread<T, DPT, KIND, 4>), g, dim3(256), 0, st, t, dp, t0, span, scale, p.kp, p.Mr,
                           ranges, nsub, rsub, p.L2, p.L2p, make_fastdiv((uint32_t)p.L2), grid, grid_stride);
    else if (p.tile <= 2048)
        hipLaunchKernelGGL((k_spread<T, DPT, KIND, 8>), g, dim3(256), 0, st, t, dp, t0, span, scale, p.kp, p.Mr,
                           ranges, nsub, rsub, p.L2, p.L2p, make_fastdiv((uint32_t)p.L2), grid, grid_stride);
    else
        hipLaunchKernelGGL((k_spread<T, DPT, KIND, 16>), g, dim3(256), 0, st, t, dp, t0, span, scale, p.kp,
                           p.Mr, ranges, nsub, rsub, p.L2, p.L2p, make_fastdiv((uint32_t)p.L2), grid, grid_stride);
}

template <typename T, typename DPT>
static void launch_spread_k(const Plan& p, int s_count, const double* t, const DPT* dp, double t0, double t_end,
                            const int64_t* ranges, int nsub, T* grid, int64_t grid_stride, hipStream_t st)
{
    if (p.kernel == MM_ES)
        launch_spread_t<T, DPT, MM_ES>(p, s_count, t, dp, t0, t_end, ranges, nsub, grid, grid_stride, st);
    else if (p.kernel == MM_GAUSSIAN)
        launch_spread_t<T, DPT, MM_GAUSSIAN>(p, s_count, t, dp, t0, t_end, ranges, nsub, grid, grid_stride, st);
    else
        launch_spread_t<T, DPT, MM_KAISER_BESSEL>(p, s_count, t, dp, t0, t_end, ranges, nsub, grid, grid_stride, st);
}

static int ilog2(int x)
{
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}

hipError_t launch_tile_ranges(const Plan& p, const int64_t* offsets, const double* t, int32_t s_begin,
                              int32_t s_count, int tiles, int tc, double t0, double T, int64_t* ranges, hipStream_t st)
{
    const double span = T - t0;
    const int64_t nr = (int64_t)s_count * tiles * 6;
    if (nr == 0) return hipSuccess;
    const RangeJob j{offsets, t, s_begin, s_count, tiles, tc, p.Mr, p.kp.w, p.kp.hw, t0, span, (double)p.Mr / span,
                     ranges};
    prof_begin("k_tile_ranges", st);
    if (p.prec == MM_PLAIN_FP64)
        hipLaunchKernelGGL(k_tile_ranges<true>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, j);
    else
        hipLaunchKernelGGL(k_tile_ranges<false>, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, j);
    prof_end("k_tile_ranges", st);
    return hipGetLastError();
}

template <typename T>
static hipError_t nufft_tiled_t(const Plan& p, const NufftWs& w, char* ws, int32_t s_begin, int32_t s_count,
                                const int64_t* offsets, const double* t, const void* dp, int dp_fp64, double t0,
                                double T_, void* coef, int64_t ldc, hipStream_t st, const SplitOut* so,
                                bool ranges_ready)
{
    using C = typename CT<T>::type;
    T* grid = (T*)(ws + w.grid);
    const int64_t gstride = 2ll * p.L1 * p.L2p;
    // event ranges per sub-tile of kRangeCells cells, nsub per series
    const int nsub = (p.Mr + kRangeCells - 1) / kRangeCells;
    int64_t* ranges = (int64_t*)(ws + w.ranges);
    if (!ranges_ready) {
        hipError_t er = launch_tile_ranges(p, offsets, t, s_begin, s_count, nsub, kRangeCells, t0, T_, ranges, st);
        if (er != hipSuccess) return er;
    }
    // recorded under the name of the kernel that runs (the polynomial path names its
    // own, one per kernel)
    bool spread_done = false;
    if constexpr (sizeof(T) == 4) {
        if (p.poly) {
            hipError_t e = launch_spread_poly(p, s_count, t, dp, dp_fp64, t0, T_, ranges, nsub, grid, gstride, st);
            if (e != hipSuccess) return e;
            spread_done = true;
        }
    }
    if (!spread_done) {
        prof_begin("k_spread", st);
        if (dp_fp64)
            launch_spread_k<T, double>(p, s_count, t, (const double*)dp, t0, T_, ranges, nsub, grid, gstride, st);
        else
            launch_spread_k<T, float>(p, s_count, t, (const float*)dp, t0, T_, ranges, nsub, grid, gstride, st);
        prof_end("k_spread", st);
    }

    if (p.fft_ab) return launch_fft_ab(p, w, ws, s_begin, s_count, grid, gstride, coef, ldc, st, so);
    if (so) return hipErrorInvalidValue;   // the split is fused only into the two-pass FFT
    const int cbs = ilog2(p.CB);
    const size_t lds1 = (size_t)(p.L1 + p.CB * (p.L1 | 1)) * sizeof(C) + (size_t)((p.L1 + 3) & ~3) * 4;
    prof_begin("k_fft_cols", st);
    hipLaunchKernelGGL(k_fft_cols<T>, dim3((p.L2 + p.CB - 1) / p.CB, s_count), dim3(256), lds1, st, grid, gstride,
                       p.L1, p.L2, p.L2p, cbs, p.F1, (const C*)(ws + w.tw1), (const C*)(ws + w.twL),
                       (const int*)(ws + w.rev1));
    prof_end("k_fft_cols", st);

    const int rs = ilog2(p.R);
    const int P = p.L1 / 2 + 1;
    const size_t lds2 = (size_t)(p.L2 + 2 * p.R * (p.L2 | 1)) * sizeof(C) + (size_t)((p.L2 + 3) & ~3) * 4;
    prof_begin("k_fft_rows", st);
    hipLaunchKernelGGL(k_fft_rows<T>, dim3((P + p.R - 1) / p.R, s_count), dim3(256), lds2, st, grid, gstride, p.L1,
                       p.L2, p.L2p, rs, p.F2, make_fastdiv((uint32_t)p.L2), (const C*)(ws + w.tw2), (const int*)(ws + w.pos2), (const C*)(ws + w.twM),
                       (const T*)(ws + w.dfac), p.N, (C*)coef, ldc, s_begin);
    prof_end("k_fft_rows", st);
    return hipGetLastError();
}

hipError_t launch_nufft_tiled(const Plan& p, const NufftWs& w, char* ws, int32_t s_begin, int32_t s_count,
                              const int64_t* offsets, const double* t, const void* dp, int dp_fp64, double t0,
                              double T, void* coef, int64_t ldc, hipStream_t st, const SplitOut* so, bool ranges_ready)
{
    if (s_count <= 0) return hipSuccess;
    if (p.prec == MM_MIXED)
        return nufft_tiled_t<float>(p, w, ws, s_begin, s_count, offsets, t, dp, dp_fp64, t0, T, coef, ldc, st, so,
                                    ranges_ready);
    if (so) return hipErrorInvalidValue;
    return nufft_tiled_t<double>(p, w, ws, s_begin, s_count, offsets, t, dp, dp_fp64, t0, T, coef, ldc, st, nullptr,
                                 ranges_ready);
}



}  // namespace mm
