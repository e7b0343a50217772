// Host-only check of the NUFFT planner (mm_plan.cpp), built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_abi.py.  It plans every
// combination of cutoff, kernel, tolerance, precision and tuning below (valid and
// invalid), checks what each accepted plan promises (Sec. 2.2.5: grid length,
// FFT split, spreading width, error estimate within tol, polynomial fit within
// tol/20, LDS of the chosen kernels within their budgets) and lays out the
// workspace for several batch sizes.  Exit status: number of failed checks.
#include <math.h>
#include <stdio.h>

#include "mm_internal.h"
#include "mm_layout.h"

using namespace mm;

static int g_fail = 0;
#define CHECK(cond, ...)                                                   \
    do {                                                                   \
        if (!(cond)) {                                                     \
            ++g_fail;                                                      \
            if (g_fail <= 20) {                                            \
                printf("FAIL %s: ", #cond);                                \
                printf(__VA_ARGS__);                                       \
                printf("\n");                                              \
            }                                                              \
        }                                                                  \
    } while (0)

static bool smooth235(long n)
{
    for (int q : {2, 3, 5})
        while (n % q == 0) n /= q;
    return n == 1;
}

static void check_plan(const Plan& p, int N, int kernel, double tol, int prec, const mm_tuning* t)
{
    const char* kn = kernel == MM_ES ? "es" : (kernel == MM_KAISER_BESSEL ? "kb" : "gauss");
    const double sg = p.sigma;
    CHECK(p.N == N && p.M == 2 * N + 1, "N %d", N);
    CHECK(p.Mr % 2 == 0 && smooth235(p.Mr), "Mr %d not even 2,3,5-smooth (N %d %s)", p.Mr, N, kn);
    CHECK(p.Mr >= (long)ceil(sg * p.M - 1e-9) && p.Mr >= 2 * p.kp.w, "Mr %d < sigma M (N %d sigma %g)", p.Mr, N, sg);
    CHECK(p.L == p.Mr / 2 && (long)p.L1 * p.L2 == p.L, "L %d != L1 %d x L2 %d", p.L, p.L1, p.L2);
    CHECK(p.kp.w >= 2 && p.kp.w <= kMaxTaps, "width %d", p.kp.w);
    CHECK(isfinite(p.est_err) && p.est_err >= 0, "est_err %g", p.est_err);
    const bool auto_width = !t || t->width == 0;
    if (auto_width && prec == MM_MIXED)
        CHECK(p.est_err <= tol * (1 + 1e-12), "est_err %g > tol %g (N %d %s w %d sigma %g poly %d)", p.est_err, tol, N,
              kn, p.kp.w, sg, p.poly);
    if (p.poly) {
        CHECK(prec == MM_MIXED && p.kp.w <= kMaxPolyTaps, "poly at w %d", p.kp.w);
        const int d0 = poly_degree_for_width(p.kp.w);
        CHECK(p.pp.deg == d0 || (d0 == kPolyDegTop && p.pp.deg == kPolyDegLow), "poly degree %d at w %d", p.pp.deg,
              p.kp.w);
        // the width's own degree fits within tol/20; the lower one only within the estimate's headroom
        if (p.pp.deg == d0) CHECK(p.poly_err <= 0.05 * tol, "poly_err %g > tol/20 (tol %g)", p.poly_err, tol);
        else CHECK(p.est_err <= tol * (1 + 1e-12), "degree %d: est_err %g > tol %g", p.pp.deg, p.est_err, tol);
        for (int j = 0; j < kMaxPolyTaps; ++j)
            for (int k = p.pp.deg + 1; k <= kMaxPolyDeg; ++k)
                CHECK(p.pp.c[j][k] == 0.f, "coefficient %d of tap %d above degree %d", k, j, p.pp.deg);
    }
    if (p.fft_ab) {
        CHECK((long)p.A1 * p.B1 == p.L1 && (long)p.A2 * p.B2 == p.L2, "codelet split %dx%d %dx%d of %d %d", p.A1, p.B1,
              p.A2, p.B2, p.L1, p.L2);
        CHECK(fft_ab_lds_cols(p) <= 64 * 1024 && fft_ab_lds_rows(p) <= 64 * 1024, "two-pass LDS %zu %zu",
              fft_ab_lds_cols(p), fft_ab_lds_rows(p));
        CHECK(p.CC >= 1 && p.RR >= 1, "CC %d RR %d", p.CC, p.RR);
    }
    CHECK(p.mom_density == 0.0 || (p.poly && p.kp.w <= 17), "moments without polynomials (w %d)", p.kp.w);
    if (p.fused) {
        CHECK(p.Mr <= kFusedMaxCells && fused_lds_bytes(p) <= kFusedMaxLds, "fused plan Mr %d LDS %zu", p.Mr,
              fused_lds_bytes(p));
        CHECK(p.poly && p.fft_ab && p.prec == MM_MIXED, "fused without its prerequisites");
    }
    CHECK(p.tile == 1024 || p.tile == 2048 || p.tile == 4096, "tile %d", p.tile);
    for (int S : {1, 7, 1000, 65535}) {
        const NufftWs w = nufft_workspace(p, S);
        const size_t parts[] = {w.tw1, w.tw2, w.twL, w.twM, w.rev1, w.pos2, w.dfac, w.flag, w.ranges, w.grid,
                                w.tLlo, w.tLhi, w.tMlo, w.tMhi};
        for (size_t o : parts) CHECK(o <= w.total && o % 256 == 0, "workspace offset %zu of %zu (S %d)", o, w.total, S);
        if (!use_fused(p, S)) CHECK(w.S_grid >= 1 && w.S_grid <= S, "S_grid %d of %d", w.S_grid, S);
    }
}

int main()
{
    const int Ns[] = {1, 2, 3, 7, 64, 100, 999, 1000, 4049, 5000, 12345, 50000, 65536, 100000, 1000000, 1 << 21};
    const int kernels[] = {MM_GAUSSIAN, MM_KAISER_BESSEL, MM_ES};
    const double tols[] = {1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10, 1e-12, 1e-14};
    const int precs[] = {MM_MIXED, MM_PLAIN_FP64};
    long plans = 0, accepted = 0;
    auto run = [&](int N, int k, double tol, int prec, const mm_tuning* t) {
        Plan p;
        const mm_status s = make_plan(N, (mm_kernel)k, tol, (mm_prec)prec, t, &p);
        ++plans;
        if (s == MM_OK) {
            ++accepted;
            check_plan(p, N, k, tol, prec, t);
        } else {
            CHECK(s == MM_ERR_ARG || s == MM_ERR_TOL || s == MM_ERR_UNSUPPORTED, "status %d", (int)s);
        }
    };
    for (int N : Ns)
        for (int k : kernels)
            for (double tol : tols)
                for (int prec : precs) run(N, k, tol, prec, nullptr);
    // tunings: oversampling, forced widths and evaluations, tiles, fused and FFT choices
    for (int N : {3, 1000, 4049, 50000})
        for (int k : kernels)
            for (double sg : {1.25, 1.55, 2.0, 2.5, 3.0})
                for (int width : {-1, 0, 4, 9, 16})
                    for (int sd : {0, 1, 2})
                        for (int tile : {0, 1024, 4096})
                            for (int fz : {-1, 0, 1})
                                for (double tol : {1e-4, 1e-6}) {
                                    const double md = fz == 1 ? 2.5 : (fz == -1 ? -1.0 : 0.0);
                                    mm_tuning t = {width, sg, tile, fz, 0.0, fz == 1, sd, 0, 0, md};
                                    run(N, k, tol, MM_MIXED, &t);
                                    if (sd == 0 && fz == 0) run(N, k, tol * 1e-4, MM_PLAIN_FP64, &t);
                                }
    // arguments the planner must refuse
    {
        Plan p;
        CHECK(make_plan(0, MM_ES, 1e-6, MM_MIXED, nullptr, &p) == MM_ERR_ARG, "N = 0 accepted");
        CHECK(make_plan((1 << 21) + 1, MM_ES, 1e-6, MM_MIXED, nullptr, &p) == MM_ERR_ARG, "N too large accepted");
        CHECK(make_plan(100, (mm_kernel)7, 1e-6, MM_MIXED, nullptr, &p) == MM_ERR_ARG, "unknown kernel accepted");
        CHECK(make_plan(100, MM_ES, 1e-6, (mm_prec)9, nullptr, &p) == MM_ERR_ARG, "unknown precision accepted");
        CHECK(make_plan(100, MM_ES, nan(""), MM_MIXED, nullptr, &p) == MM_ERR_TOL, "NaN tol accepted");
        CHECK(make_plan(100, MM_ES, 1e-7, MM_MIXED, nullptr, &p) == MM_ERR_TOL, "mixed tol below 1e-6 accepted");
        CHECK(make_plan(100, MM_ES, 0.5, MM_PLAIN_FP64, nullptr, &p) == MM_ERR_TOL, "tol 0.5 accepted");
        mm_tuning t = {0, 1.0, 0, 0, 0.0, 0, 0, 0, 0, 0.0};
        CHECK(make_plan(100, MM_ES, 1e-6, MM_MIXED, &t, &p) == MM_ERR_ARG, "sigma 1 accepted");
        t.sigma = 0.0;
        t.width = kMaxTaps + 2;
        CHECK(make_plan(100, MM_ES, 1e-6, MM_MIXED, &t, &p) == MM_ERR_ARG, "width above the maximum accepted");
    }
    printf("%ld plans, %ld accepted, %d failed checks\n", plans, accepted, g_fail);
    return g_fail > 255 ? 255 : g_fail;
}
