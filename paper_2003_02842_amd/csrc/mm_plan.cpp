// Host-side planning of a type-1 NUFFT: spreading width from the tolerance,
// oversampled grid length, two-pass FFT factorisation, kernel shape constants.
// Pure host code: no device calls, so it can be exercised without a GPU.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "mm_internal.h"

namespace mm {

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
    if (tune && tune->width > 0) {
        w = tune->width;
        if (kernel == MM_GAUSSIAN) { if (w & 1) ++w; msp = w / 2; }
        else if (kernel == MM_KAISER_BESSEL) { if (!(w & 1)) ++w; msp = (w - 1) / 2; }
        else msp = (w + 1) / 2;
    }
    if (w < 2 || w > kMaxTaps || msp < 1) return MM_ERR_ARG;
    p->msp = msp;

    KernParams& kp = p->kp;
    kp.kind = kernel;
    kp.w = w;
    kp.hw = 0.5 * w;
    if (kernel == MM_ES) {
        double bpt = (tune && tune->es_beta_per_tap > 0) ? tune->es_beta_per_tap : 2.3;
        kp.es_beta = bpt * w;              // beta = 2.3 omega, support +-omega/2 cells (Eq. Der:10-11)
        kp.es_inv_hw = 2.0 / w;
    } else if (kernel == MM_GAUSSIAN) {
        kp.g_lambda = sg * msp / (sg - 0.5);   // step I.3 of the FGG algorithm
        kp.g_t1 = kPi / kp.g_lambda;
        kp.g_msp = msp;
        for (int k = 0; k <= msp; ++k) kp.g_e3[k] = exp(-kp.g_t1 * k * k);
    } else {
        kp.kb_b = kPi * (2.0 - 1.0 / sg);      // b of Eq. Der:9
        kp.kb_m = msp;
        kp.kb_inv_norm = msp / sinh(kp.kb_b * msp);
    }

    // Oversampled grid: even, 2,3,5-smooth, >= sigma M and >= 2 w (the grid
    // must be longer than the spreading width).
    uint64_t target = (uint64_t)ceil(sg * p->M - 1e-9);
    target = std::max<uint64_t>(target, 2ull * w);
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
    if (!make_fft_desc(L1, &p->F1) || !make_fft_desc(L2, &p->F2)) return MM_ERR_UNSUPPORTED;

    const size_t cs = (prec == MM_MIXED) ? 8 : 16;    // bytes per complex value
    const size_t budget = 64 * 1024;
    int CB = 16;
    while (CB > 1 && (size_t)(CB * (L1 | 1) + L1) * cs > budget) CB >>= 1;
    while (CB > 1 && CB / 2 >= L2) CB >>= 1;      // stays a power of two
    p->CB = CB;
    int R = 8;
    int P = L1 / 2 + 1;                          // row pairs (k1, L1 - k1), k1 = 0..L1/2
    while (R > 1 && (size_t)(2 * R * (L2 | 1) + L2) * cs > budget) R >>= 1;
    while (R > 1 && R / 2 >= P) R >>= 1;         // stays a power of two
    p->R = R;
    int tile = (prec == MM_MIXED) ? 2048 : 1024;
    if (tune && tune->tile > 0) tile = tune->tile <= 1024 ? 1024 : (tune->tile <= 2048 ? 2048 : 4096);
    p->tile = tile;
    p->fused = 0;
    p->fused_threads = 256;
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
    w.flag = o; o += 256;
    w.S_grid = (p.prec == MM_MIXED && !p.fused) ? S : (p.fused ? 0 : 1);
    const size_t tiles = (size_t)(p.Mr + p.tile - 1) / p.tile;
    w.ranges = o; o += al(8 * 6 * tiles * (size_t)w.S_grid);
    w.grid = o; o += al(rs * (size_t)p.Mr * (size_t)w.S_grid);
    w.total = o;
    return w;
}

}  // namespace mm
