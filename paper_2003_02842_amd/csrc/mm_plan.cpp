// Host-side planning of a type-1 NUFFT: spreading width from the tolerance,
// oversampled grid length, two-pass FFT factorisation, kernel shape constants.
// Pure host code: no device calls, so it can be exercised without a GPU.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "mm_internal.h"
#include "mm_layout.h"

namespace mm {

// LDS budget of one FFT workgroup and the largest row-pair block of the row pass.
#ifndef MM_FFT_LDS_MAX
#define MM_FFT_LDS_MAX (64 * 1024)
#endif
#ifndef MM_FFT_RR_MAX
#define MM_FFT_RR_MAX 4
#endif

static const double kPi = 3.14159265358979323846264338327950288;

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    f.M = ((1ull << 42) + d - 1) / d;
    return f;
}

static bool is_235_smooth(uint64_t n)
{
    if (n == 0) return false;
    for (uint64_t p : {2ull, 3ull, 5ull})
        while (n % p == 0) n /= p;
    return n == 1;
}

uint64_t smooth_even_at_least(uint64_t n)
{
    uint64_t m = n < 2 ? 2 : n;
    if (m & 1) ++m;
    while (!is_235_smooth(m)) m += 2;
    return m;
}

// Radix sequence of an in-LDS DIF FFT of length n: fours first, then fives,
// threes and a final two.
static bool make_fft_desc(int n, FFTDesc* F)
{
    memset(F, 0, sizeof(*F));
    F->n = n;
    int rad[kMaxStages * 2];
    int ns = 0, x = n;
    while (x % 4 == 0) { rad[ns++] = 4; x /= 4; }
    while (x % 5 == 0) { rad[ns++] = 5; x /= 5; }
    while (x % 3 == 0) { rad[ns++] = 3; x /= 3; }
    while (x % 2 == 0) { rad[ns++] = 2; x /= 2; }
    if (x != 1 || ns > kMaxStages) return false;
    F->ns = ns;
    int len = n;
    for (int s = 0; s < ns; ++s) {
        F->r[s] = rad[s];
        F->m[s] = len / rad[s];
        F->tws[s] = n / len;
        F->dm[s] = make_fastdiv((uint32_t)F->m[s]);
        F->dnr[s] = make_fastdiv((uint32_t)(n / rad[s]));
        len = F->m[s];
    }
    // pair consecutive stages into register-resident double passes
    F->np = 0;
    for (int s = 0; s < ns; s += 2) {
        const int q = F->np++;
        const bool dbl = s + 1 < ns;
        const int span = F->m[s] * F->r[s];
        F->p1[q] = F->r[s];
        F->p2[q] = dbl ? F->r[s + 1] : 1;
        F->plen[q] = span;
        F->pm1[q] = F->m[s];
        F->pm2[q] = dbl ? F->m[s + 1] : F->m[s];
        F->pts1[q] = n / span;
        F->pts2[q] = dbl ? n / F->m[s] : 1;
        F->pdtask[q] = make_fastdiv((uint32_t)(n / (F->p1[q] * F->p2[q])));
        F->pdm2[q] = make_fastdiv((uint32_t)F->pm2[q]);
    }
    return true;
}

// Split L = L1 * L2 with L1 <= L2, both <= kMaxSub, L1 as close to sqrt(L) as possible.
static bool split_len(int64_t L, int* L1, int* L2)
{
    int best = -1;
    for (int64_t a = 1; a * a <= L; ++a)
        if (L % a == 0 && L / a <= kMaxSub) best = (int)a;
    if (best < 0) return false;
    *L1 = best;
    *L2 = (int)(L / best);
    return true;
}

void gauss_legendre_pos(int n_pos, double* x, double* w)
{
    // Newton iteration on the Legendre polynomial P_n, n = 2 n_pos, from the
    // classical initial guess cos(pi (i - 1/4)/(n + 1/2)); P_n and P_n' by the
    // three-term recurrence.
    int n = 2 * n_pos;
    for (int i = 0; i < n_pos; ++i) {
        double z = cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// ------------------------------------------------------------------ error estimate
// The kernel as the spreading taps evaluate it (cells; taps cover (-hw, hw]).
static double host_psi(const KernParams& kp, double x)
{
    if (kp.kind == MM_ES) {
        double z = x * kp.es_inv_hw;
        return exp(kp.es_beta * (sqrt(std::max(1.0 - z * z, 0.0)) - 1.0));
    }
    if (kp.kind == MM_GAUSSIAN) return exp(-kp.g_t1 * x * x);
    double s2 = kp.kb_m * kp.kb_m - x * x;
    double v;
    if (s2 > 0) { double q = sqrt(s2); v = sinh(kp.kb_b * q) / q; }
    else if (s2 < 0) { double q = sqrt(-s2); v = sin(kp.kb_b * q) / q; }
    else v = kp.kb_b;
    return v * kp.kb_inv_norm;
}

// Interpolate tap j, as a function of s = f - 1/2 in [-1/2, 1/2], at the deg+1
// Chebyshev points, solve for monomial coefficients (partial pivoting), round them
// to FP32 and return the largest deviation from the kernel over the interval.
// The kernel is even, so tap w-1-j is tap j at -s: only taps j < ceil(w/2) are fitted.
static double fit_poly(const KernParams& kp, int deg, PolyParams* pp)
{
    pp->deg = deg;
    double worst = 0.0;
    for (int j = 0; j < kMaxPolyTaps; ++j)
        for (int k = 0; k <= kMaxPolyDeg; ++k) pp->c[j][k] = 0.f;
    const int n = deg + 1;
    for (int j = 0; j < (kp.w + 1) / 2; ++j) {
        double A[kMaxPolyDeg + 1][kMaxPolyDeg + 2];
        for (int m = 0; m < n; ++m) {
            const double sm = 0.5 * cos(kPi * (m + 0.5) / n);
            double pw = 1.0;
            for (int k = 0; k < n; ++k) { A[m][k] = pw; pw *= sm; }
            A[m][n] = host_psi(kp, j + 0.5 - sm - kp.hw);
        }
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int r = col + 1; r < n; ++r)
                if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
            for (int k = 0; k <= n; ++k) std::swap(A[col][k], A[piv][k]);
            for (int r = 0; r < n; ++r) {
                if (r == col) continue;
                const double fct = A[r][col] / A[col][col];
                for (int k = col; k <= n; ++k) A[r][k] -= fct * A[col][k];
            }
        }
        for (int k = 0; k < n; ++k) pp->c[j][k] = (float)(A[k][n] / A[k][k]);
        for (int q = 0; q <= 200; ++q) {
            const double sq = -0.5 + q / 200.0;
            double acc = pp->c[j][deg], mir = pp->c[j][deg];
            for (int k = deg - 1; k >= 0; --k) {
                acc = acc * sq + pp->c[j][k];
                mir = mir * -sq + pp->c[j][k];
            }
            worst = std::max(worst, fabs(acc - host_psi(kp, j + 0.5 - sq - kp.hw)));
            worst = std::max(worst, fabs(mir - host_psi(kp, (kp.w - 1 - j) + 0.5 - sq - kp.hw)));
        }
    }
    return worst;
}

static double host_i0(double x)
{
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int j = 1; j < 1000; ++j) {
        term *= q / ((double)j * (double)j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// Fourier transform at nu (cycles per cell) of the kernel truncated to the taps'
// support: 2 int_0^hw psi(x) cos(2 pi nu x) dx, composite 16-point Gauss-Legendre.
static double host_psihat_trunc(const KernParams& kp, double nu)
{
    struct Rule {
        double x[8], w[8];
        Rule() { gauss_legendre_pos(8, x, w); }
    };
    static const Rule rule;   // built once, thread-safe (C++11 function-local static)
    const double* gx = rule.x;
    const double* gw = rule.w;
    const int panels = 32;
    const double h = kp.hw / panels;
    double tot = 0.0;
    for (int q = 0; q < panels; ++q) {
        const double c = (q + 0.5) * h, r = 0.5 * h;
        for (int i = 0; i < 8; ++i)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                double x = c + sgn * r * gx[i];
                tot += r * gw[i] * host_psi(kp, x) * cos(2.0 * kPi * nu * x);
            }
    }
    return 2.0 * tot;
}

// What the deconvolution divides by (same formulas as the device factors).
static double host_psihat_deconv(const KernParams& kp, double nu)
{
    if (kp.kind == MM_GAUSSIAN) return sqrt(kp.g_lambda) * exp(-kPi * kp.g_lambda * nu * nu);
    if (kp.kind == MM_KAISER_BESSEL) {
        double a = kp.kb_b * kp.kb_b - (2.0 * kPi * nu) * (2.0 * kPi * nu);
        return kPi * kp.kb_inv_norm * host_i0(kp.kb_m * sqrt(std::max(a, 0.0)));
    }
    struct Rule {
        double x[kGLNodes], w[kGLNodes];
        Rule() { gauss_legendre_pos(kGLNodes, x, w); }
    };
    static const Rule rule;   // built once, thread-safe
    const double* gx = rule.x;
    const double* gw = rule.w;
    double acc = 0.0;
    for (int q = 0; q < kGLNodes; ++q)
        acc += gw[q] * exp(kp.es_beta * (sqrt(1.0 - gx[q] * gx[q]) - 1.0)) * cos(2.0 * kPi * nu * kp.hw * gx[q]);
    return 2.0 * kp.hw * acc;
}

// Worst-case relative error of a coefficient, over k in [0, N]: the aliased
// images sum_{m != 0} |psi_hat(k/Mr + m)| of the truncated kernel (Poisson
// summation of the periodic grid, Eqs. Der:14-16) plus the mismatch between the
// truncated kernel's transform and the factor the deconvolution divides by,
// both relative to that factor.  Bounds the l2 error of Eq. Der:18.
static double estimate_error_uncached(const KernParams& kp, int Mr, int N)
{
    double worst = 0.0;
    const int samples = 17;
    for (int i = 0; i < samples; ++i) {
        const double k = (double)N * i / (samples - 1);
        const double nu = k / Mr;
        const double den = host_psihat_deconv(kp, nu);
        double ali = 0.0;
        for (int m = 1; m <= 3; ++m)
            ali += fabs(host_psihat_trunc(kp, nu + m)) + fabs(host_psihat_trunc(kp, nu - m));
        const double mis = fabs(host_psihat_trunc(kp, nu) - den);
        worst = std::max(worst, (ali + mis) / fabs(den));
    }
    return worst;
}

// FP32 rounding on the mixed path.  The spread grid and its transform carry
// relative errors of a few units of u = 2^-24, and the deconvolution (Eq. Der:17)
// multiplies the error at frequency k by psi_hat(0) / psi_hat(k / Mr), which
// grows quickly as sigma falls towards 1.  For a flat spectrum the relative l2
// error of the coefficients is u G rms_k psi_hat(0) / psi_hat(k / Mr); G was
// measured against the FP64 oracle over sigma = 1.25..2.5 (ES,
// Gaussian and Kaiser-Bessel, uneven series up to 4 events per cell): 1.2-2.2
// with per-tap polynomials, 3.6-4.2 with the ES formula, 4.5-6.0 with the
// Gaussian formula and 6.5-9.8 with the Kaiser-Bessel formula.
static double rounding_gain(int kernel, bool poly)
{
    if (poly) return 3.0;   // per-event taps 2.0; the per-cell moment form up to 1.5x that
    if (kernel == MM_KAISER_BESSEL) return 10.0;
    return kernel == MM_GAUSSIAN ? 6.5 : 4.5;
}

static double rounding_error(const KernParams& kp, int Mr, int N, double gain)
{
    const int samples = 65;
    const double d0 = host_psihat_deconv(kp, 0.0);
    double acc = 0.0;
    for (int i = 0; i < samples; ++i) {
        const double r = d0 / host_psihat_deconv(kp, (double)N * i / (samples - 1) / Mr);
        acc += r * r;
    }
    return 0x1p-24 * gain * sqrt(acc / samples);
}

static std::mutex g_est_mu;
static std::map<std::tuple<int, int, long long, long long, int, int, int>, double> g_est_cache;

// Aliasing and truncation (a worst case over k, well above the l2 error they
// cause), or the FP32 rounding term when `gain` > 0 (the mixed path) and it is
// larger.
static double estimate_error(const KernParams& kp, double sigma, int Mr, int N, double gain)
{
    auto key = std::make_tuple(kp.kind, kp.w, (long long)llround(sigma * 1e6), (long long)llround(kp.es_beta * 1e6),
                               Mr, N, (int)llround(gain * 1000));
    {
        std::lock_guard<std::mutex> lk(g_est_mu);
        auto it = g_est_cache.find(key);
        if (it != g_est_cache.end()) return it->second;
    }
    double e = estimate_error_uncached(kp, Mr, N);
    if (gain > 0) e = std::max(e, rounding_error(kp, Mr, N, gain));
    std::lock_guard<std::mutex> lk(g_est_mu);
    g_est_cache[key] = e;
    return e;
}

// Kernel shape for a width w (taps per event) at oversampling sg.
static void set_kernel(KernParams& kp, int kernel, int w, int msp, double sg, const mm_tuning* tune)
{
    memset(&kp, 0, sizeof(kp));
    kp.kind = kernel;
    kp.w = w;
    kp.hw = 0.5 * w;
    if (kernel == MM_ES) {
        // beta = 2.3 omega at sigma = 2 (Eq. Der:10-11); other sigma scale it by (1 - 1/(2 sigma)) / (3/4)
        double bpt = (tune && tune->es_beta_per_tap > 0) ? tune->es_beta_per_tap : 2.3 * (1.0 - 0.5 / sg) / 0.75;
        kp.es_beta = bpt * w;
        kp.es_inv_hw = 2.0 / w;
    } else if (kernel == MM_GAUSSIAN) {
        kp.g_lambda = sg * msp / (sg - 0.5);   // step I.3 of the FGG algorithm
        kp.g_t1 = kPi / kp.g_lambda;
        kp.g_msp = msp;
        for (int k = 0; k <= msp && k <= kMaxTaps / 2; ++k) kp.g_e3[k] = exp(-kp.g_t1 * k * k);
    } else {
        kp.kb_b = kPi * (2.0 - 1.0 / sg);      // b of Eq. Der:9
        kp.kb_m = msp;
        kp.kb_inv_norm = msp / sinh(kp.kb_b * msp);
    }
}

// Oversampled grid: even, 2,3,5-smooth, >= sigma M and >= 2 w (the grid must be
// longer than the spreading width), and splittable into two in-LDS sub-FFTs.
static mm_status set_grid(Plan* p)
{
    uint64_t target = (uint64_t)ceil(p->sigma * p->M - 1e-9);
    target = std::max<uint64_t>(target, 2ull * p->kp.w);
    target = std::max<uint64_t>(target, 8ull);
    uint64_t Mr = smooth_even_at_least(target);
    int L1 = 0, L2 = 0;
    while (true) {
        if (Mr / 2 > (uint64_t)kMaxSub * kMaxSub) return MM_ERR_UNSUPPORTED;
        if (split_len((int64_t)(Mr / 2), &L1, &L2)) break;
        Mr = smooth_even_at_least(Mr + 2);
    }
    p->Mr = (int)Mr;
    p->L = (int)(Mr / 2);
    p->L1 = L1;
    p->L2 = L2;
    return MM_OK;
}

static int msp_for_width(int kernel, int w)
{
    if (kernel == MM_GAUSSIAN) return w / 2;
    if (kernel == MM_KAISER_BESSEL) return (w - 1) / 2;
    return (w + 1) / 2;
}

// Codelet split n = A x B (A <= B <= max_codelet, smallest B) of a two-pass
// codelet FFT, and the LDS of its column and row passes.
bool fft_ab_split(int n, int max_codelet, int* A, int* B)
{
    static const int sizes[] = {1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 18, 20, 24, 25, 27, 30, 32};
    int best = -1;
    for (int a : sizes)
        for (int b : sizes)
            if (a * b == n && a <= b && b <= max_codelet && (best < 0 || b < best)) {
                best = b;
                *A = a;
                *B = b;
            }
    return best > 0;
}

size_t fft_ab_lds_cols(const Plan& p)
{
    const size_t cs = p.prec == MM_MIXED ? 8 : 16;
    return cs * ((size_t)p.L1 + (1u << p.tw_lo_bits) + p.tw_hi_L + (size_t)p.A1 * (p.B1 * p.CC + 1));
}

size_t fft_ab_lds_rows(const Plan& p)
{
    const size_t cs = p.prec == MM_MIXED ? 8 : 16;
    return cs * ((size_t)p.L2 + (1u << p.tw_lo_bits) + p.tw_hi_M + 2 * (size_t)p.RR * (p.L2 + 1));
}

// LDS of the fused kernel's spreading buffers at width w (the widths it is built for)
static size_t fused_spread_bytes(int w)
{
    switch (w) {
#define MM_SB(n) case n: return SpreadLds<n, kFusedPPT, kFusedThreads, kFusedEV>::bytes;
        MM_SB(4) MM_SB(5) MM_SB(6) MM_SB(7) MM_SB(8) MM_SB(9) MM_SB(10) MM_SB(11) MM_SB(12)
#undef MM_SB
    }
    return (size_t)1 << 30;
}

// Dynamic LDS of k_nufft_fused: the tables, then the larger of the grid plus
// exchange buffer and the spreading's buffers (which lie over them).
size_t fused_lds_bytes(const Plan& p)
{
    const FusedLds f = fused_lds(p.L1, p.L2, p.A1, p.B1, p.tw_lo_bits, p.tw_hi_L);
    return std::max(8 * (size_t)f.total, 8 * (size_t)f.z + fused_spread_bytes(p.kp.w));
}

// Whether the fused kernel can run this plan: the mixed path with per-tap
// polynomials of 4 to 12 taps (the widths compiled here), the two-pass codelet
// FFT with sub-lengths of at most 16 points, a grid of at most kFusedMaxCells, and
// its LDS within kFusedMaxLds.
bool fused_fits(const Plan& p)
{
    if (p.prec != MM_MIXED || !p.poly || !p.fft_ab || p.Mr > kFusedMaxCells || p.kp.w < 4 || p.kp.w > 12)
        return false;
    if (p.B1 > 16 || p.B2 > 16) return false;   // codelets of the fused kernel: up to 16 points
    if (p.tw_hi_L != p.tw_hi_M) return false;
    return fused_lds_bytes(p) <= kFusedMaxLds;
}


mm_status make_plan(int32_t N, mm_kernel kernel, double tol, mm_prec prec, const mm_tuning* tune, Plan* p)
{
    memset(p, 0, sizeof(*p));
    if (N < 1 || N > (1 << 21)) return MM_ERR_ARG;
    if (kernel != MM_GAUSSIAN && kernel != MM_KAISER_BESSEL && kernel != MM_ES) return MM_ERR_ARG;
    if (prec != MM_PLAIN_FP64 && prec != MM_MIXED) return MM_ERR_ARG;
    if (!(tol == tol)) return MM_ERR_TOL;
    double tmin = (prec == MM_MIXED) ? 1e-6 : 1e-14;
    if (tol < tmin * (1 - 1e-12) || tol > 0.1 * (1 + 1e-12)) return MM_ERR_TOL;

    p->prec = prec;
    p->kernel = kernel;
    p->N = N;
    p->M = 2 * N + 1;
    p->tol = tol;
    p->sigma = (tune && tune->sigma > 0) ? tune->sigma : 2.0;
    if (p->sigma < 1.25 || p->sigma > 8.0) return MM_ERR_ARG;
    const double sg = p->sigma;

    // Spreading half-width rules of Sec. 2.2.5.  The digit count guards the
    // ceiling at exact powers of ten.
    int digits = (int)ceil(-log10(tol) - 1e-9);
    int msp, w;
    if (kernel == MM_GAUSSIAN) {
        msp = (int)floor(-log(tol) * (sg - 0.5) / (kPi * (sg - 1.0)) + 0.5);
        if (msp < 1) msp = 1;
        w = 2 * msp;                       // taps -(M_sp-1)..M_sp around the cell (FGG)
    } else if (kernel == MM_KAISER_BESSEL) {
        msp = (digits + 2) / 2;
        w = 2 * msp + 1;                   // taps -M_sp..M_sp
    } else {
        msp = (digits + 2) / 2 + 2;
        w = 2 * msp;                       // support +-M_sp cells
    }
    p->msp = msp;
    const int req = tune ? tune->width : 0;
    const int sd = tune ? tune->spread_direct : 0;
    const bool want_poly = sd == 2 || (sd == 0 && kernel != MM_GAUSSIAN);
    if (req > 0) {
        w = req;
        if (kernel == MM_GAUSSIAN && (w & 1)) ++w;
        if (kernel == MM_KAISER_BESSEL && !(w & 1)) ++w;
        msp = msp_for_width(kernel, w);
    } else if (req == 0 && (prec == MM_MIXED || (kernel != MM_GAUSSIAN && sg != 2.0))) {
        // smallest width whose worst-case error estimate meets tol (the FP64
        // path keeps the rules above at sigma = 2, the oversampling they are
        // stated for; the Gaussian's rule already carries sigma)
        const int step = (kernel == MM_ES) ? 1 : 2;
        int wa = (kernel == MM_KAISER_BESSEL) ? 3 : 2;
        bool found = false;
        for (; wa <= kMaxTaps; wa += step) {
            Plan q = *p;
            int ma = msp_for_width(kernel, wa);
            if (ma < 1) continue;
            set_kernel(q.kp, kernel, wa, ma, sg, tune);
            if (set_grid(&q) != MM_OK) continue;
            // with per-tap polynomials their fit (admitted up to tol/20, below) takes
            // its share of the bound
            const bool pc = prec == MM_MIXED && want_poly && wa <= kMaxPolyTaps;
            const double gain = (prec == MM_MIXED) ? rounding_gain(kernel, pc) : 0.0;
            if (estimate_error(q.kp, sg, q.Mr, N, gain) + (pc ? 0.05 * tol : 0.0) <= tol) { found = true; break; }
        }
        if (!found) return MM_ERR_TOL;   // tol out of reach at this oversampling
        w = wa;
        msp = msp_for_width(kernel, w);
    }
    if (w < 2 || w > kMaxTaps || msp < 1) return MM_ERR_ARG;
    p->wmsp = msp;
    set_kernel(p->kp, kernel, w, msp, sg, tune);
    mm_status gs = set_grid(p);
    if (gs != MM_OK) return gs;
    {
        const int q = (prec == MM_MIXED) ? 16 : 8;   // complex values per 128 bytes
        p->L2p = (p->L2 + q - 1) / q * q;
    }
    if (!make_fft_desc(p->L1, &p->F1) || !make_fft_desc(p->L2, &p->F2)) return MM_ERR_UNSUPPORTED;
    const int L1 = p->L1, L2 = p->L2;

    const size_t cs = (prec == MM_MIXED) ? 8 : 16;    // bytes per complex value
    const size_t budget = 64 * 1024;
    int CB = 16;
    while (CB > 1 && (size_t)(CB * (L1 | 1) + L1) * cs + (size_t)((L1 + 3) & ~3) * 4 > budget) CB >>= 1;
    while (CB > 1 && CB / 2 >= L2) CB >>= 1;      // stays a power of two
    p->CB = CB;
    int R = 8;
    int P = L1 / 2 + 1;                          // row pairs (k1, L1 - k1), k1 = 0..L1/2
    while (R > 1 && (size_t)(2 * R * (L2 | 1) + L2) * cs + (size_t)((L2 + 3) & ~3) * 4 > budget) R >>= 1;
    while (R > 1 && R / 2 >= P) R >>= 1;         // stays a power of two
    p->R = R;
    // two-pass sub-transforms with register codelets when both lengths split
    {
        const int maxc = 32;
        p->fft_ab = fft_ab_split(L1, maxc, &p->A1, &p->B1) && fft_ab_split(L2, maxc, &p->A2, &p->B2);
        if (tune && tune->fft_generic == 1) p->fft_ab = 0;
        int bits = 0;
        while ((1ll << (2 * bits)) < (long long)p->L) ++bits;
        p->tw_lo_bits = bits;
        p->tw_hi_L = (int)((p->L + (1 << bits) - 1) >> bits);
        p->tw_hi_M = p->tw_hi_L;
        p->CC = (prec == MM_MIXED) ? 16 : 8;      // 128-byte row segments
        while (p->CC > 1 && p->CC / 2 >= L2) p->CC >>= 1;
        const size_t lds_max = MM_FFT_LDS_MAX;
        p->RR = MM_FFT_RR_MAX;                     // a power of two
        while (p->RR > 1 && (fft_ab_lds_rows(*p) > lds_max || 2 * p->RR * std::max(p->A2, p->B2) > 512)) p->RR >>= 1;
        while (p->RR > 1 && p->RR / 2 >= L1 / 2 + 1) p->RR >>= 1;
        while (p->fft_ab && p->CC > 1 && fft_ab_lds_cols(*p) > lds_max) p->CC >>= 1;
        if (p->fft_ab && (fft_ab_lds_rows(*p) > 64 * 1024 || fft_ab_lds_cols(*p) > 64 * 1024)) p->fft_ab = 0;
    }
    // FP32 spreading from per-tap polynomials when they stay well inside tol.  By
    // default for Kaiser-Bessel (its sinh/sin formula is the costliest per tap) and
    // ES (2.7 vs 2.9-3.2 ms on the large universe, and closer to FP64); the Gaussian
    // needs wider kernels, whose longer tap records make the formula faster there
    // (3.6 vs 4.8 ms).
    p->poly = 0;
    p->poly_err = 0.0;
    if (prec == MM_MIXED && p->kp.w <= kMaxPolyTaps && want_poly) {
        const double err = fit_poly(p->kp, poly_degree_for_width(p->kp.w), &p->pp);
        if (err <= 0.05 * tol) {
            p->poly = 1;
            p->poly_err = err;
        }
    }
    // the polynomials' own deviation from the kernel (relative to its peak, 1) adds to the bound
    const double est_kernel =
        estimate_error(p->kp, sg, p->Mr, N, (prec == MM_MIXED) ? rounding_gain(kernel, p->poly) : 0.0);
    // one degree less (one FMA per tap pair and one moment per key fewer) where its
    // fit still leaves the whole estimate within tol
    if (p->poly && p->pp.deg == kPolyDegTop) {
        PolyParams low;
        const double err = fit_poly(p->kp, kPolyDegLow, &low);
        if (est_kernel + err <= tol) {
            p->pp = low;
            p->poly_err = err;
        }
    }
    p->est_err = est_kernel + (p->poly ? p->poly_err : 0.0);
    int tile = (prec == MM_MIXED) ? 2048 : 1024;
    if (tune && tune->tile > 0) tile = tune->tile <= 1024 ? 1024 : (tune->tile <= 2048 ? 2048 : 4096);
    p->tile = tile;
    // dense tiles from per-cell moments (the per-tap polynomials' coefficients, up to 17 taps)
    {
        const double md = tune ? tune->moment_density : 0.0;
        p->mom_density = (p->poly && p->kp.w <= 17 && md >= 0.0) ? (md > 0.0 ? md : kMomDensity) : 0.0;
    }
    // the fused single-workgroup NUFFT of small grids: 0 (auto) for calls of at least
    // kFusedMinSeries series, 1 for any call, -1 never
    const int fz = tune ? tune->fused : 0;
    p->fused = (fz >= 0 && fused_fits(*p)) ? 1 : 0;
    p->fused_min_series = fz == 1 ? 1 : kFusedMinSeries;
    return MM_OK;
}

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

NufftWs nufft_workspace(const Plan& p, int32_t S)
{
    NufftWs w;
    const size_t rs = (p.prec == MM_MIXED) ? 4 : 8;   // bytes per real value
    size_t o = 0;
    w.tw1 = o;  o += al(2 * rs * p.L1);
    w.tw2 = o;  o += al(2 * rs * p.L2);
    w.twL = o;  o += al(2 * rs * (size_t)p.L);
    w.twM = o;  o += al(2 * rs * (size_t)p.L);
    w.rev1 = o; o += al(4 * (size_t)p.L1);
    w.pos2 = o; o += al(4 * (size_t)p.L2);
    w.dfac = o; o += al(rs * (size_t)(p.N + 1));
    w.tLlo = o; o += al(2 * rs * ((size_t)1 << p.tw_lo_bits));
    w.tLhi = o; o += al(2 * rs * (size_t)p.tw_hi_L);
    w.tMlo = o; o += al(2 * rs * ((size_t)1 << p.tw_lo_bits));
    w.tMhi = o; o += al(2 * rs * (size_t)p.tw_hi_M);
    w.flag = o; o += 256;
    const bool fused = use_fused(p, S);
    w.S_grid = fused ? 0 : (p.prec == MM_MIXED ? S : 1);
    const size_t tiles = (size_t)(p.Mr + kRangeCells - 1) / kRangeCells;   // event-range sub-tiles
    w.ranges = o; o += al(8 * 6 * (fused ? (size_t)S : tiles * (size_t)w.S_grid));
    w.grid = o; o += al(rs * 2 * (size_t)p.L1 * (size_t)p.L2p * (size_t)w.S_grid);
    w.total = o;
    return w;
}

}  // namespace mm
