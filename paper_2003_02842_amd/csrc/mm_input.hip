// Paper-form input: n x D price and time matrices with NaN where an asset has no
// observation (inputs of the MM algorithm), turned into the CSR returns that the
// NUFFT takes (steps F.1-F.3), with the time window of the time-rescaling
// algorithm (global min and max of the times) and the Nyquist cutoffs of the
// Nyquist-frequency algorithm, N_i = floor((t_max - t_min) / (2 dt_i)) with dt_i
// the smallest gap between consecutive observation times of asset i and
// N = min_i N_i.
//
//   k_in_count    per asset: valid observations, min and max time, bad prices
//   k_in_offsets  one workgroup: exclusive scans of valid counts and return counts
//   k_in_compact  per asset: valid times and log prices, in order, to the workspace
//   k_in_returns  per return: t_h, log p_{h+1} - log p_h, the gap t_{h+1} - t_h
//   k_in_nyquist  one workgroup: per-asset cutoffs and their minimum
#include <hip/hip_runtime.h>

#include "mm_internal.h"

namespace mm {

// Flags of the data check (host turns any of them into MM_ERR_DATA).
enum : int { kBadPrice = 1, kUnsorted = 2, kRepeated = 4 };

__device__ __forceinline__ bool valid_obs(double p, double t) { return isfinite(p) && isfinite(t); }

__device__ __forceinline__ void atomic_min_pos(double* a, double v)
{
    // positive doubles order like their bit patterns
    atomicMin((unsigned long long*)a, (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(256) void k_in_count(int64_t n, const double* __restrict__ P, const double* __restrict__ Tm,
                                                  int64_t ld, int64_t* __restrict__ cnt, double* __restrict__ tmin,
                                                  double* __restrict__ tmax, int* __restrict__ flag)
{
    __shared__ int64_t sc[256];
    __shared__ double smn[256], smx[256];
    const int i = blockIdx.x;
    const double* p = P + (int64_t)i * ld;
    const double* tt = Tm + (int64_t)i * ld;
    int64_t c = 0;
    double mn = INFINITY, mx = -INFINITY;
    int bad = 0;
    for (int64_t h = threadIdx.x; h < n; h += 256) {
        const double ph = p[h], th = tt[h];
        if (valid_obs(ph, th)) {
            ++c;
            mn = fmin(mn, th);
            mx = fmax(mx, th);
            if (!(ph > 0.0)) bad |= kBadPrice;
        }
    }
    sc[threadIdx.x] = c;
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sc[threadIdx.x] += sc[threadIdx.x + s];
            smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + s]);
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (bad) atomicOr(flag, bad);
    if (threadIdx.x == 0) {
        cnt[i] = sc[0];
        tmin[i] = smn[0];
        tmax[i] = smx[0];
    }
}

// Exclusive scans over assets: voff (valid observations) and roff (returns,
// max(count - 1, 0)); meta[0] = total returns, meta[1] = total valid; window =
// (min, max) over assets with any observation.
__global__ __launch_bounds__(1024) void k_in_offsets(int D, const int64_t* __restrict__ cnt,
                                                     const double* __restrict__ tmin, const double* __restrict__ tmax,
                                                     int64_t* __restrict__ voff, int64_t* __restrict__ roff,
                                                     int64_t* __restrict__ meta, double* __restrict__ window)
{
    __shared__ int64_t sv[1024], sr[1024];
    __shared__ double smn[1024], smx[1024];
    int64_t carry_v = 0, carry_r = 0;
    double mn = INFINITY, mx = -INFINITY;
    for (int base = 0; base < D; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int64_t c = i < D ? cnt[i] : 0;
        sv[threadIdx.x] = c;
        sr[threadIdx.x] = c > 0 ? c - 1 : 0;
        if (i < D && c > 0) {
            mn = fmin(mn, tmin[i]);
            mx = fmax(mx, tmax[i]);
        }
        __syncthreads();
        // Hillis-Steele inclusive scan
        for (int s = 1; s < 1024; s <<= 1) {
            int64_t a = 0, b = 0;
            if ((int)threadIdx.x >= s) {
                a = sv[threadIdx.x - s];
                b = sr[threadIdx.x - s];
            }
            __syncthreads();
            sv[threadIdx.x] += a;
            sr[threadIdx.x] += b;
            __syncthreads();
        }
        if (i < D) {
            voff[i] = carry_v + sv[threadIdx.x] - c;
            roff[i] = carry_r + sr[threadIdx.x] - (c > 0 ? c - 1 : 0);
        }
        carry_v += sv[1023];
        carry_r += sr[1023];
        __syncthreads();
    }
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + s]);
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        voff[D] = carry_v;
        roff[D] = carry_r;
        meta[0] = carry_r;
        meta[1] = carry_v;
        window[0] = smn[0];
        window[1] = smx[0];
    }
}

// Valid observations of asset i, in row order, to tv/lv at voff[i] (chunked
// block scan of the valid flags).
__global__ __launch_bounds__(256) void k_in_compact(int64_t n, const double* __restrict__ P,
                                                    const double* __restrict__ Tm, int64_t ld,
                                                    const int64_t* __restrict__ voff, double* __restrict__ tv,
                                                    double* __restrict__ lv)
{
    __shared__ int s[256];
    const int i = blockIdx.x;
    const double* p = P + (int64_t)i * ld;
    const double* tt = Tm + (int64_t)i * ld;
    int64_t pos = voff[i];
    for (int64_t h0 = 0; h0 < n; h0 += 256) {
        const int64_t h = h0 + threadIdx.x;
        double ph = 0.0, th = 0.0;
        int v = 0;
        if (h < n) {
            ph = p[h];
            th = tt[h];
            v = valid_obs(ph, th) ? 1 : 0;
        }
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int a = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        if (v) {
            const int64_t q = pos + s[threadIdx.x] - 1;
            tv[q] = th;
            lv[q] = log(ph);
        }
        pos += s[255];
        __syncthreads();
    }
}

// One thread per return h of asset i (binary search of the asset over roff).
__global__ void k_in_returns(int D, const int64_t* __restrict__ voff, const int64_t* __restrict__ roff,
                             const double* __restrict__ tv, const double* __restrict__ lv, double* __restrict__ t,
                             void* __restrict__ dp, int dp_fp64, double* __restrict__ mindt, int* __restrict__ flag)
{
    const int64_t E = roff[D];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= E) return;
    int lo = 0, hi = D;   // last asset with roff <= r
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (roff[mid] <= r) lo = mid;
        else hi = mid;
    }
    while (lo + 1 < D && roff[lo + 1] <= r) ++lo;   // skip assets without returns
    const int64_t j = r - roff[lo];
    const int64_t q = voff[lo] + j;
    const double t0 = tv[q], t1 = tv[q + 1];
    t[r] = t0;
    const double d = __dsub_rn(lv[q + 1], lv[q]);
    if (dp_fp64) ((double*)dp)[r] = d;
    else ((float*)dp)[r] = (float)d;
    const double gap = __dsub_rn(t1, t0);
    if (!(gap >= 0.0)) atomicOr(flag, kUnsorted);
    else if (gap == 0.0) atomicOr(flag, kRepeated);
    else atomic_min_pos(&mindt[lo], gap);
}

__global__ __launch_bounds__(1024) void k_in_nyquist(int D, const int64_t* __restrict__ cnt,
                                                     const double* __restrict__ mindt,
                                                     const double* __restrict__ window, int32_t* __restrict__ nyq,
                                                     int32_t* __restrict__ nmin)
{
    __shared__ int32_t sm[1024];
    const double span = __dsub_rn(window[1], window[0]);
    int32_t m = INT32_MAX;
    for (int i = threadIdx.x; i < D; i += 1024) {
        int32_t Ni = INT32_MAX;
        if (cnt[i] >= 2 && mindt[i] < INFINITY) {
            const double x = floor(__ddiv_rn(span, __dmul_rn(2.0, mindt[i])));
            Ni = x >= (double)INT32_MAX ? INT32_MAX : (int32_t)x;
        }
        nyq[i] = Ni;
        m = min(m, Ni);
    }
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = min(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *nmin = sm[0];
}

__global__ void k_in_init(int D, double* mindt, int* flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < D) mindt[i] = INFINITY;
    if (i == 0) *flag = 0;
}

// The zero-padded FFT method (appendix) moves every time to the nearest of Nstar
// equally spaced points of [t0, T): l = round(u Nstar), u = (t - t0)/(T - t0),
// l = Nstar wrapping to 0.
__global__ void k_snap(int64_t E, const double* __restrict__ t, double t0, double span, int64_t Nstar,
                       double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    const double u = __ddiv_rn(__dsub_rn(t[i], t0), span);
    int64_t l = (int64_t)rint(__dmul_rn(u, (double)Nstar));
    if (l >= Nstar) l -= Nstar;
    out[i] = __dadd_rn(t0, __dmul_rn(span, __ddiv_rn((double)l, (double)Nstar)));
}

hipError_t launch_snap(int64_t E, const double* t, double t0, double T, int64_t Nstar, double* out, hipStream_t st)
{
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_snap, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, E, t, t0, T - t0, Nstar, out);
    return hipGetLastError();
}

InputWs input_workspace(int64_t n, int32_t D)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    InputWs w;
    size_t o = 0;
    w.cnt = o;   o += al(8 * (size_t)D);
    w.tmin = o;  o += al(8 * (size_t)D);
    w.tmax = o;  o += al(8 * (size_t)D);
    w.mindt = o; o += al(8 * (size_t)D);
    w.voff = o;  o += al(8 * ((size_t)D + 1));
    w.meta = o;  o += al(64);
    w.tv = o;    o += al(8 * (size_t)n * (size_t)D);
    w.lv = o;    o += al(8 * (size_t)n * (size_t)D);
    w.total = o;
    return w;
}

hipError_t launch_input(int64_t n, int32_t D, const double* P, const double* Tm, int64_t ld, int64_t* offsets,
                        double* t, void* dp, int dp_fp64, int32_t* nyq, const InputWs& w, char* ws, hipStream_t st)
{
    int64_t* cnt = (int64_t*)(ws + w.cnt);
    double* tmin = (double*)(ws + w.tmin);
    double* tmax = (double*)(ws + w.tmax);
    double* mindt = (double*)(ws + w.mindt);
    int64_t* voff = (int64_t*)(ws + w.voff);
    int64_t* meta = (int64_t*)(ws + w.meta);        // [0] returns, [1] valid, [2] flag, [3] N, [4..5] window
    int* flag = (int*)(meta + 2);
    int32_t* nmin = (int32_t*)(meta + 3);
    double* window = (double*)(meta + 4);
    prof_begin("k_in_count", st);
    hipLaunchKernelGGL(k_in_init, dim3((D + 255) / 256), dim3(256), 0, st, D, mindt, flag);
    hipLaunchKernelGGL(k_in_count, dim3(D), dim3(256), 0, st, n, P, Tm, ld, cnt, tmin, tmax, flag);
    hipLaunchKernelGGL(k_in_offsets, dim3(1), dim3(1024), 0, st, D, cnt, tmin, tmax, voff, offsets, meta, window);
    hipLaunchKernelGGL(k_in_compact, dim3(D), dim3(256), 0, st, n, P, Tm, ld, voff, (double*)(ws + w.tv),
                       (double*)(ws + w.lv));
    prof_end("k_in_count", st);
    return hipGetLastError();
}

hipError_t launch_input_returns(int32_t D, int64_t E, int64_t* offsets, double* t, void* dp, int dp_fp64,
                                int32_t* nyq, const InputWs& w, char* ws, hipStream_t st)
{
    int64_t* cnt = (int64_t*)(ws + w.cnt);
    double* mindt = (double*)(ws + w.mindt);
    int64_t* voff = (int64_t*)(ws + w.voff);
    int64_t* meta = (int64_t*)(ws + w.meta);
    int* flag = (int*)(meta + 2);
    int32_t* nmin = (int32_t*)(meta + 3);
    double* window = (double*)(meta + 4);
    if (E > 0)
        hipLaunchKernelGGL(k_in_returns, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, D, voff, offsets,
                           (const double*)(ws + w.tv), (const double*)(ws + w.lv), t, dp, dp_fp64, mindt, flag);
    hipLaunchKernelGGL(k_in_nyquist, dim3(1), dim3(1024), 0, st, D, cnt, mindt, window, nyq, nmin);
    return hipGetLastError();
}

}  // namespace mm
