/*
 * Plain FP64 CPU oracle for the Malliavin-Mancino Fourier estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or constant with the GPU
 * library.
 *
 * What it computes (Chang, Pienaar, Gebbie, "Malliavin-Mancino estimators
 * implemented with non-uniform fast Fourier transforms"):
 *
 *  - Rescaling (time-rescaling algorithm, appendix): the paper maps times to
 *    [0, 2pi] with tilde t = 2pi (t - tmin)/(tmax - tmin).  Here the window
 *    [t0, T) is explicit: u = (t - t0)/(T - t0) in [0,1) and tilde t = 2pi u.
 *    u == 1 folds to 0 (the transform is 2pi-periodic).
 *
 *  - Fourier coefficients of the returns (Sec. 2.2, the equation defining
 *    F(dp_i)(k)):  c_k = (1/2pi) sum_h delta_h exp(-i k tilde t_h),
 *    evaluated directly for every requested k (the "for-loop" method,
 *    appendix algorithm MS).  The phase k*u is split exactly into an integer
 *    and a fraction (p = k*u rounded, e = fma(k,u,-p) its exact error) so the
 *    angle 2pi*frac(k u) is accurate to ~1e-16 rad for any k; sin/cos come
 *    from the C library in double precision; the sum over events is
 *    Neumaier-compensated.
 *
 *  - Dirichlet and Fejer estimators (Sec. 2.1, Eqs. Der:2 and Der:3; the
 *    convolution step C.1/C.2 of the MM algorithm):
 *        Sigma_ij = sum_{|s|<=N} w_s (2pi)^2 c_s^(i) conj(c_s^(j))
 *    with w_s = 1/(2N+1) (Dirichlet) or w_s = (1 - |s|/N)/(N+1) (Fejer,
 *    exactly as printed in Eq. Der:3).  The (2pi)^2 undoes the 1/2pi of each
 *    coefficient, so Sigma equals the double sum over events of Eq. Der:2/3.
 *    orc_cov_full sums s = -N..N with complex arithmetic from coefficients
 *    computed at every s; orc_cov uses the Hermitian symmetry
 *    c_{-s} = conj(c_s) of real returns (Sec. 2.2.2) and sums s = 0..N.
 *
 *  - Correlation (MM algorithm, last step): R_ij = Sigma_ij/sqrt(Sigma_ii Sigma_jj),
 *    NaN where a variance is not positive.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double rescale(double t, double t0, double T)
{
    double u = (t - t0) / (T - t0);
    if (u >= 1.0) u -= 1.0;
    return u;
}

/* Neumaier (improved Kahan) compensated accumulation. */
static void neumaier_add(double* sum, double* comp, double x)
{
    double s = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - s) + x;
    else                       *comp += (x - s) + *sum;
    *sum = s;
}

/* Coefficients of one series for k = klo..khi: out[2*(k-klo)] = Re, [..+1] = Im. */
static void coeffs_series(int64_t n, const double* u, const double* dp,
                          int64_t k, double* re_out, double* im_out)
{
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    double kd = (double)k;
    for (int64_t h = 0; h < n; ++h) {
        double p = kd * u[h];
        double e = fma(kd, u[h], -p);        /* k*u == p + e exactly */
        double f = (p - floor(p)) + e;       /* phase in cycles, mod 1 */
        double ang = TWO_PI * f;
        neumaier_add(&sr, &cr, dp[h] * cos(ang));
        neumaier_add(&si, &ci, -dp[h] * sin(ang));
    }
    *re_out = (sr + cr) / TWO_PI;
    *im_out = (si + ci) / TWO_PI;
}

/* c_k, k = klo..khi, for one series of n events. */
void orc_coeffs(int64_t n, const double* t, const double* dp, double t0, double T,
                int64_t klo, int64_t khi, double* out)
{
    double* u = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t h = 0; h < n; ++h) u[h] = rescale(t[h], t0, T);
    int64_t nk = khi - klo + 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nk; ++j)
        coeffs_series(n, u, dp, klo + j, &out[2 * j], &out[2 * j + 1]);
    free(u);
}

/* c_k of one series of n events at the nk listed frequencies ks[] (any order). */
void orc_coeffs_at(int64_t n, const double* t, const double* dp, double t0, double T,
                   const int64_t* ks, int64_t nk, double* out)
{
    double* u = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t h = 0; h < n; ++h) u[h] = rescale(t[h], t0, T);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < nk; ++j)
        coeffs_series(n, u, dp, ks[j], &out[2 * j], &out[2 * j + 1]);
    free(u);
}

/* S series in CSR form; coef is S x ldc complex (interleaved re,im), k = 0..N. */
void orc_coeffs_batch(int32_t S, const int64_t* offsets, const double* t, const double* dp,
                      double t0, double T, int32_t N, double* coef, int64_t ldc)
{
    int64_t E = offsets[S];
    double* u = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    for (int64_t h = 0; h < E; ++h) u[h] = rescale(t[h], t0, T);
    int64_t nk = (int64_t)N + 1;
#pragma omp parallel for schedule(dynamic, 8) collapse(2)
    for (int32_t s = 0; s < S; ++s)
        for (int64_t k = 0; k < nk; ++k) {
            int64_t a = offsets[s], b = offsets[s + 1];
            coeffs_series(b - a, u + a, dp + a, k,
                          &coef[2 * (s * ldc + k)], &coef[2 * (s * ldc + k) + 1]);
        }
    free(u);
}

static double weight(int64_t s, int32_t N, int32_t basis)
{
    int64_t a = s < 0 ? -s : s;
    if (basis == 0) return 1.0 / (2.0 * N + 1.0);                     /* Dirichlet */
    return (1.0 - (double)a / (double)N) / ((double)N + 1.0);          /* Fejer as printed */
}

static void correlation(int32_t D, const double* cov, double* corr)
{
    for (int32_t i = 0; i < D; ++i)
        for (int32_t j = 0; j < D; ++j) {
            double a = cov[i * D + i], b = cov[j * D + j];
            corr[i * D + j] = (a > 0.0 && b > 0.0) ? cov[i * D + j] / (sqrt(a) * sqrt(b)) : NAN;
        }
}

/* Full-range form: coef_full is S x ldc complex holding s = -N..N at columns
 * 0..2N.  Writes Re and Im of Sigma for G groups of D series (G x D x D). */
void orc_cov_full(int32_t G, int32_t D, const double* coef_full, int64_t ldc, int32_t N,
                  int32_t basis, double* cov_re, double* cov_im, double* corr)
{
#pragma omp parallel for collapse(3)
    for (int32_t g = 0; g < G; ++g)
        for (int32_t i = 0; i < D; ++i)
            for (int32_t j = 0; j < D; ++j) {
                const double* ci = coef_full + 2 * ((int64_t)(g * D + i) * ldc);
                const double* cj = coef_full + 2 * ((int64_t)(g * D + j) * ldc);
                double sr = 0, cr = 0, si = 0, cim = 0;
                for (int64_t s = -N; s <= N; ++s) {
                    int64_t c = s + N;
                    double w = weight(s, N, basis) * TWO_PI * TWO_PI;
                    double ar = ci[2 * c], ai = ci[2 * c + 1];
                    double br = cj[2 * c], bi = -cj[2 * c + 1];     /* conj */
                    neumaier_add(&sr, &cr, w * (ar * br - ai * bi));
                    neumaier_add(&si, &cim, w * (ar * bi + ai * br));
                }
                cov_re[((int64_t)g * D + i) * D + j] = sr + cr;
                cov_im[((int64_t)g * D + i) * D + j] = si + cim;
            }
    if (corr)
        for (int32_t g = 0; g < G; ++g)
            correlation(D, cov_re + (int64_t)g * D * D, corr + (int64_t)g * D * D);
}

/* Symmetric form from k = 0..N (coef is S x ldc complex, column k = c_k):
 * Sigma_ij = (2pi)^2 [w_0 c_0^i conj c_0^j + 2 sum_{k=1..N} w_k Re(c_k^i conj c_k^j)].
 * One result per cutoff in Ns (nN of them): cov is nN x G x D x D. */
void orc_cov(int32_t G, int32_t D, const double* coef, int64_t ldc, const int32_t* Ns,
             int32_t nN, int32_t basis, double* cov, double* corr)
{
#pragma omp parallel for collapse(4)
    for (int32_t q = 0; q < nN; ++q)
        for (int32_t g = 0; g < G; ++g)
            for (int32_t i = 0; i < D; ++i)
                for (int32_t j = 0; j < D; ++j) {
                    int32_t N = Ns[q];
                    const double* ci = coef + 2 * ((int64_t)(g * D + i) * ldc);
                    const double* cj = coef + 2 * ((int64_t)(g * D + j) * ldc);
                    double sum = 0, comp = 0;
                    for (int64_t k = 0; k <= N; ++k) {
                        double re = ci[2 * k] * cj[2 * k] + ci[2 * k + 1] * cj[2 * k + 1];
                        double mult = (k == 0) ? 1.0 : 2.0;
                        neumaier_add(&sum, &comp, mult * weight(k, N, basis) * re);
                    }
                    cov[(((int64_t)q * G + g) * D + i) * D + j] = TWO_PI * TWO_PI * (sum + comp);
                }
    if (corr)
        for (int64_t m = 0; m < (int64_t)nN * G; ++m)
            correlation(D, cov + m * D * D, corr + m * D * D);
}
