/*
 * mm.h -- C ABI of the MI355X (gfx950) Malliavin-Mancino covariance library.
 *
 * The estimator (Chang, Pienaar, Gebbie, "Malliavin-Mancino estimators
 * implemented with non-uniform fast Fourier transforms") has two stages:
 *
 *   1. mm_nufft1: the Fourier coefficients of each series' returns
 *        c_k = (1/2pi) sum_h delta_h exp(-i k tilde t_h),  k = 0..N
 *      (Sec. 2.2, the equation defining F(dp_i)(k)), computed by a type-1
 *      non-uniform FFT (Sec. 2.2.5, Eqs. Der:14-17): spread the events onto an
 *      oversampled periodic grid with a Gaussian (Eqs. Der:5, 7), Kaiser-Bessel
 *      (Eqs. Der:8-9) or exponential of semicircle (Eqs. Der:10-11) kernel, FFT
 *      the grid, divide by the kernel's Fourier transform.  Negative k follow from c_{-k} = conj(c_k) (real
 *      returns, Sec. 2.2.2) and are not stored.
 *
 *   2. mm_cov: the Dirichlet (Eq. Der:2) or Fejer (Eq. Der:3) estimate
 *        Sigma_ij = (2pi)^2 sum_{|k|<=N} w_k c_k^(i) conj(c_k^(j))
 *      with w_k = 1/(2N+1) or (1-|k|/N)/(N+1) (the Fejer weights exactly as
 *      printed in Eq. Der:3 and step C.2 of the MM algorithm), and the
 *      correlation R_ij = Sigma_ij / sqrt(Sigma_ii Sigma_jj) (MM algorithm,
 *      last step).  Several cutoffs N can be evaluated from one coefficient set
 *      because c_k does not depend on N.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (gfx950 global memory) owned by the
 *     caller, except where marked "host".  The library keeps no pointer after
 *     it returns and never frees caller memory.
 *   - `stream` is a hipStream_t (NULL: the default stream).  Work is enqueued
 *     asynchronously on it; results are ready when the stream reaches them.
 *   - Arguments that the host can check are checked before anything is
 *     launched; on error nothing is enqueued and the status says why.
 *   - Nothing throws across this boundary.  Device failures map to MM_ERR_HIP.
 *   - One process may call from several host threads on different streams;
 *     calls sharing a workspace buffer must be ordered by the caller.
 */
#ifndef MM_H_
#define MM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MM_OK = 0,
    MM_ERR_ARG = 1,          /* a size, pointer or enum argument is invalid */
    MM_ERR_DATA = 2,         /* validate=1 found unsorted, out-of-window or non-finite events */
    MM_ERR_TOL = 3,          /* tol outside [1e-14,1e-1] (FP64) or [1e-6,1e-1] (mixed), or
                                out of reach at the requested oversampling */
    MM_ERR_WORKSPACE = 4,    /* ws_bytes below the size the *_workspace_size call reports */
    MM_ERR_HIP = 5,          /* a HIP runtime call failed */
    MM_ERR_UNSUPPORTED = 6   /* a valid request the library does not implement */
} mm_status;

typedef enum { MM_DIRICHLET = 0, MM_FEJER = 1 } mm_basis;            /* Eq. Der:2 / Eq. Der:3 */
typedef enum { MM_GAUSSIAN = 0, MM_KAISER_BESSEL = 1, MM_ES = 2 } mm_kernel;  /* Eqs. Der:5 / 8-9 / 10-11 */
typedef enum {
    MM_PLAIN_FP64 = 0,       /* FP64 everywhere, one launch chain per series, FP64 contraction */
    MM_MIXED = 1             /* FP64 time reduction and deconvolution factors; FP32 spreading, FFT and
                                coefficients; contraction on BF16 MFMA with hi/lo split, FP32 accumulate */
} mm_prec;

/* Optional overrides of the planner (an autotuner's output).  Zero means "let
 * the planner choose"; pass NULL for all defaults. */
typedef struct {
    int32_t width;             /* taps per event (>= 2, <= 40); 0: MM_MIXED picks the smallest width whose
                                  a-priori error estimate meets tol, MM_PLAIN_FP64 uses the paper's rule;
                                  -1: the paper's rule for both */
    double sigma;              /* oversampling factor of the grid, >= 1.25 */
    int32_t tile;              /* cells per spreading tile (tiled path) */
    int32_t fused;             /* the fused small-grid NUFFT (MM_MIXED, per-tap polynomials of 4-12 taps, grids of
                                  at most 8192 cells): one workgroup per series spreads into LDS, runs both FFT
                                  passes there and writes only c_k.  0 (auto): taken for calls of at least 64
                                  series; 1: for any call it can run; -1: never (the tiled kernels) */
    double es_beta_per_tap;    /* ES shape: beta = es_beta_per_tap * width (paper: 2.3) */
    int32_t fft_generic;       /* 1: run the grid FFT with the generic in-LDS radix passes even where both
                                  sub-lengths split into register codelets (0: auto) */
    int32_t spread_direct;     /* MM_MIXED spreading: 1 evaluates the kernel formula at every (event, cell)
                                  pair; 2 uses per-tap polynomials (fitted within tol/20) evaluated once per
                                  event; 0 (auto): polynomials for Kaiser-Bessel and ES, the formula for the
                                  Gaussian */
    int32_t syrk_tile;         /* MM_MIXED contraction on MFMA (D(D+1)/2 > 1024): output tile edge, 128 or 256;
                                  0: the built-in model (256 for large D and long k ranges) */
    int32_t syrk_splits;       /* ... and the number of k-ranges each tile's sum is split into (partial tiles
                                  summed afterwards), >= 1, at most one per 32 real columns; 0: the model */
    double moment_density;     /* MM_MIXED spreading with per-tap polynomials: grid tiles holding at least this
                                  many events per cell are spread from per-cell moments (sum_d c_jd M_l[d],
                                  M_l[d] the sum of v s^d over the events starting at cell l), the others by
                                  per-event taps; 0: the default (3.0), < 0: per-event taps everywhere */
} mm_tuning;

/* What the planner chose (host only, no device work). */
typedef struct {
    int32_t N;                 /* cutoff */
    int32_t width;             /* taps per event */
    int32_t msp;               /* spreading half-width M_sp of the paper's rule (Sec. 2.2.5) */
    int32_t Mr;                /* oversampled grid length (even, 2,3,5-smooth, >= sigma (2N+1)) */
    int32_t L1, L2;            /* Mr/2 = L1 * L2 (two-pass complex FFT) */
    int32_t fused;             /* 1 if the fused small-grid NUFFT can run this plan (mm_tuning.fused) */
    int32_t tile;              /* spreading tile of the tiled path */
    double sigma;              /* oversampling factor used in the kernel shape rules */
    double beta;               /* ES beta, Gaussian lambda or Kaiser-Bessel b */
    double tol;
    double est_err;            /* a-priori bound on the relative coefficient error: aliasing of the truncated
                                  kernel plus deconvolution mismatch (worst case over k); on the mixed path the
                                  FP32 rounding term 2^-24 G rms_k psi_hat(0)/psi_hat(k/Mr) instead when larger
                                  (G measured per evaluation: 2 polynomials, 4.5 ES, 6.5 Gaussian, 10
                                  Kaiser-Bessel formula), plus the per-tap polynomials' largest deviation
                                  from the kernel where they are used */
} mm_plan_info;

/* Plan of a type-1 NUFFT of cutoff N (Sec. 2.2.5): the spreading width follows
 * the paper's tolerance rules (Sec. 2.2.5, with the ES rule's M_sp + 2) on the
 * FP64 path at sigma = 2 (and for the Gaussian, whose rule carries sigma), and
 * otherwise is the smallest width whose a-priori estimate (est_err) meets tol; the
 * grid is Mr = smallest even 2,3,5-smooth length >= max(sigma(2N+1), 2 width, 8)
 * with sigma = 2 (Sec. 2.2.5), unless `tune` overrides.  MM_ERR_TOL also when
 * no width up to 40 meets tol at the requested sigma.  Host only. */
mm_status mm_plan_query(int32_t N, mm_kernel kernel, double tol, mm_prec prec,
                        const mm_tuning* tune, mm_plan_info* out /* host */);

/* Bytes of device workspace mm_nufft1 needs for S series. */
mm_status mm_nufft1_workspace_size(int32_t S, int32_t N, mm_kernel kernel, double tol, mm_prec prec,
                                   const mm_tuning* tune, size_t* bytes /* host */);

/* Type-1 NUFFT of S series (Sec. 2.2.5; coefficients of the equation defining
 * F(dp_i)(k), Sec. 2.2).
 *   offsets  int64[S+1], CSR: series s owns events offsets[s] .. offsets[s+1]-1
 *            (offsets[0] = 0, nondecreasing).  A series may be empty.
 *   t        float64[E]: event times, nondecreasing within a series, in [t0, T].
 *            Rescaled as u = (t - t0)/(T - t0) and tilde t = 2 pi u (time-rescaling
 *            algorithm, appendix); u = 1 is the same point as u = 0.
 *   dp       float32[E] (dp_is_fp64 = 0) or float64[E] (dp_is_fp64 = 1): the return
 *            delta_h = p(t_{h+1}) - p(t_h) attached to t_h (left endpoint).
 *   N        cutoff >= 1; coefficients k = 0..N are produced.
 *   kernel, tol, prec, tune: see the enums; tol is the target relative l2 error of
 *            each series' coefficients (Eq. Der:18).
 *   coef     S x ldc complex, row-major, ldc >= N+1: float2 (MM_MIXED) or double2
 *            (MM_PLAIN_FP64); column k holds c_k including the 1/2pi factor.
 *   ws       device workspace of at least mm_nufft1_workspace_size bytes (256-byte aligned).
 *   validate 1: check the events on the device first (sorted, inside [t0, T], finite),
 *            which synchronises `stream` and returns MM_ERR_DATA on failure; 0: the
 *            result for such data is undefined.
 * Errors: MM_ERR_ARG (S < 0, N < 1, T <= t0, non-finite t0/T, ldc < N+1, NULL
 * pointers), MM_ERR_TOL, MM_ERR_WORKSPACE, MM_ERR_DATA, MM_ERR_HIP. */
mm_status mm_nufft1(int32_t S, const int64_t* offsets, const double* t, const void* dp, int32_t dp_is_fp64,
                    double t0, double T, int32_t N, mm_kernel kernel, double tol, mm_prec prec,
                    const mm_tuning* tune, void* coef, int64_t ldc, void* ws, size_t ws_bytes,
                    int32_t validate, void* stream);

/* Bytes of device workspace mm_cov needs (may be 0); `tune` as for mm_cov. */
mm_status mm_cov_workspace_size(int32_t G, int32_t D, int32_t Nmax, int32_t nN, mm_prec prec,
                                const mm_tuning* tune, size_t* bytes /* host */);

/* Dirichlet or Fejer estimates (Eqs. Der:2, Der:3; MM algorithm steps C.1/C.2)
 * and correlations (MM algorithm, last step) for G groups of D consecutive
 * series, for each cutoff in Ns.
 *   coef     (G*D) x ldc complex as written by mm_nufft1 (float2 for MM_MIXED,
 *            double2 for MM_PLAIN_FP64), columns k = 0..max(Ns).
 *   Ns       host int32[nN], each in 1..ldc-1, 1 <= nN <= 128.
 *   cov      nN x G x D x D, row-major: float (MM_MIXED) or double (MM_PLAIN_FP64).
 *   corr     same shape and type, or NULL.  R_ij is NaN where Sigma_ii <= 0 or
 *            Sigma_jj <= 0 (an empty series).
 *   tune     NULL, or the contraction's tile and k-split (mm_tuning.syrk_tile, syrk_splits;
 *            the other fields are ignored here)
 * All cutoffs come from one pass over k where that costs less than a product per
 * cutoff: small D by FP64 running sums; on the MFMA path (mixed, large D) from
 * Gram matrices of the k-segments between consecutive cutoffs, summed in k order
 * (Dirichlet from one product; Fejer from two, the second weighted by N_j - k
 * within each segment j, so that every cutoff's weights (N - k)/(N(N+1)) come
 * from non-negative combinations), taken when max(Ns) (twice it for Fejer) is
 * below the sum of the distinct cutoffs and there are at most 64 of them.
 * Errors: MM_ERR_ARG, MM_ERR_WORKSPACE, MM_ERR_UNSUPPORTED, MM_ERR_HIP. */
mm_status mm_cov(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ns, int32_t nN,
                 mm_basis basis, mm_prec prec, const mm_tuning* tune, void* cov, void* corr, void* ws,
                 size_t ws_bytes, void* stream);

/* Bytes of device workspace mm_estimate needs for G*D series and the cutoffs Ns
 * (host int32[nN]): room for the coefficients at k = 0..max(Ns), the NUFFT
 * workspace and the contraction workspace. */
mm_status mm_estimate_workspace_size(int32_t G, int32_t D, const int32_t* Ns, int32_t nN, mm_kernel kernel,
                                     double tol, mm_prec prec, const mm_tuning* tune, size_t* bytes /* host */);

/* Both stages in one call: the coefficients of all G*D series at N = max(Ns)
 * (as mm_nufft1, without validation) and the estimates at every cutoff in Ns (as
 * mm_cov).  One NUFFT serves every cutoff because c_k does not depend on N
 * (Sec. 2.2, equation defining F(dp_i)(k)); Monte Carlo replicates are the G
 * groups (Sec. 3).
 *   coef     optional S x ldc output of the coefficients (ldc >= max(Ns)+1); NULL keeps
 *            them in ws.  With NULL, G = 1, one cutoff and D on the MFMA path (mixed,
 *            D(D+1)/2 > 1024, two-pass FFT), the coefficients are not stored at all:
 *            the FFT's row pass writes the contraction's split BF16 operands itself,
 *            one FFT row (fixed k1, coefficients k1 + L1 k2) per contiguous run of
 *            columns.  The contraction sums the same kind of products in another
 *            column order, so the results agree with the two-call form to FP32
 *            summation rounding, not bit for bit; repeated calls and graph replays
 *            are bit for bit.
 *   cov, corr  as mm_cov (corr may be NULL).
 *   ws       device workspace of at least mm_estimate_workspace_size bytes (256-byte aligned).
 *   use_graph 1: the first call with a given set of arguments (every pointer, size,
 *            scalar, the stream and the current device) records the launch sequence
 *            into a HIP graph and launches it; later calls with the same set launch
 *            the recorded graph.  The graph reads the buffers at replay time, so new
 *            data in the same buffers is picked up.  Requires a non-NULL stream (the
 *            legacy default stream cannot be captured).  At most 64 graphs are kept;
 *            recording a 65th synchronises the device and frees the oldest.
 *            0: launched directly.
 * Errors: MM_ERR_ARG, MM_ERR_TOL, MM_ERR_WORKSPACE, MM_ERR_UNSUPPORTED (G*D > 65535),
 * MM_ERR_HIP. */
mm_status mm_estimate(int32_t G, int32_t D, const int64_t* offsets, const double* t, const void* dp,
                      int32_t dp_is_fp64, double t0, double T, const int32_t* Ns, int32_t nN, mm_basis basis,
                      mm_kernel kernel, double tol, mm_prec prec, const mm_tuning* tune, void* coef, int64_t ldc,
                      void* cov, void* corr, void* ws, size_t ws_bytes, int32_t use_graph, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): mm_estimate with the
 * same arguments but no workspace argument and no graph recording (launched
 * directly, as use_graph = 0).  Its workspace is a fixed device array of
 * MM_SCRATCH_BYTES that the library holds on each GPU it runs on until the process
 * ends; the caller still passes the inputs and outputs (coef may be NULL, as
 * there).  The call allocates no device memory and records no graph.
 *   Sizes: the request's mm_estimate_workspace_size must not exceed
 *   MM_SCRATCH_BYTES (64 MiB: e.g. 100 series at N = 5000 need 19 MiB, 300 series
 *   at N = 3000 need 38 MiB), else MM_ERR_WORKSPACE before anything is launched.
 *   Sharing: every call on one GPU uses that GPU's one array, so calls that
 *   overlap in time on one GPU (different streams or host threads) race; order
 *   them.  The array keeps the last call's contents; nothing in it is read before
 *   the same call writes it.
 * Results equal mm_estimate's (same kernels) bit for bit.  Errors: as mm_estimate,
 * plus MM_ERR_WORKSPACE for a request beyond the fixed size. */
#define MM_SCRATCH_BYTES ((size_t)64 << 20)
mm_status mm_estimate_noalloc(int32_t G, int32_t D, const int64_t* offsets, const double* t, const void* dp,
                              int32_t dp_is_fp64, double t0, double T, const int32_t* Ns, int32_t nN,
                              mm_basis basis, mm_kernel kernel, double tol, mm_prec prec, const mm_tuning* tune,
                              void* coef, int64_t ldc, void* cov, void* corr, void* stream);

/* Synchronises the device and frees every graph mm_estimate recorded. */
mm_status mm_graph_cache_clear(void);

/* Bytes of device workspace mm_cov_pairwise needs (Ni: host int32[D]). */
mm_status mm_cov_pairwise_workspace_size(int32_t G, int32_t D, const int32_t* Ni, mm_prec prec,
                                         size_t* bytes /* host */);

/* Pairwise estimates with per-asset cutoffs (Sec. 3: when assets have their own
 * Nyquist cutoffs N_i, pair (i, j) is estimated at N_ij = min(N_i, N_j)):
 *   cov[g][i][j]  = the Dirichlet or Fejer estimate of pair (i, j) at N_ij
 *   corr[g][i][j] = cov_ij(N_ij) / sqrt(cov_ii(N_ij) cov_jj(N_ij)), the correlation of the
 *                  pairwise 2 x 2 estimate (NaN for a non-positive variance); may be NULL
 * The diagonal holds each asset's variance at its own N_i.  One coefficient set
 * (columns 0..max N_i) serves all pairs, with any number of distinct cutoffs: for
 * small D (D(D+1)/2 <= 1024) the estimate is swept over the distinct cutoffs and
 * each entry read from its pair's cutoff; otherwise the assets are taken in
 * ascending order of cutoff, so that a pair's cutoff is the lower-ranked asset's,
 * and one product of unweighted coefficients with coefficients weighted at each
 * asset's own cutoff gives every entry (BF16 hi/lo MFMA on MM_MIXED, FP64 tiles on
 * MM_PLAIN_FP64); the correlations take each asset's variance at every cutoff up
 * to its own from a prefix-sum table.
 *   coef   (G*D) x ldc as for mm_cov, ldc >= max N_i + 1
 *   Ni     host int32[D], each >= 1, shared by all groups
 *   cov, corr  G x D x D, float (MM_MIXED) or double (MM_PLAIN_FP64)
 * Synchronises `stream`.  The result need not be positive semi-definite.
 * Errors: MM_ERR_ARG, MM_ERR_WORKSPACE, MM_ERR_UNSUPPORTED (G or D above 65535), MM_ERR_HIP. */
mm_status mm_cov_pairwise(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ni, mm_basis basis,
                          mm_prec prec, void* cov, void* corr, void* ws, size_t ws_bytes, void* stream);

/* Result of mm_matrix_to_csr (host). */
typedef struct {
    int64_t E;                 /* returns written (CSR length) */
    int32_t N;                 /* Nyquist cutoff min_i N_i (INT32_MAX if no asset has two observations) */
    double t0, T;              /* time window: min and max observation time over all assets */
} mm_csr_info;

/* Bytes of device workspace mm_matrix_to_csr needs (two n*D FP64 staging arrays
 * plus per-asset scalars). */
mm_status mm_matrix_to_csr_workspace_size(int64_t n, int32_t D, size_t* bytes /* host */);

/* The MM algorithm's own input form (its inputs P and T; steps I.1-I.2 and
 * F.1-F.3; the time-rescaling and Nyquist-frequency algorithms): n x D matrices of
 * prices and times, column-major (column i = asset i, element (h, i) at i*ld + h,
 * ld >= n), NaN where an asset has no observation.  An observation counts when
 * both its price and its time are finite.  Writes the CSR input of mm_nufft1:
 *   offsets  int64[D+1]; asset i owns returns offsets[i] .. offsets[i+1]-1
 *   t        float64[cap]: time of the left observation of each return
 *   dp       float32 or float64[cap]: log p_{h+1} - log p_h (natural log)
 *   nyq      int32[D]: N_i = floor((t_max - t_min) / (2 dt_i)), dt_i the smallest gap between
 *            consecutive observation times of asset i (the Nyquist-frequency algorithm on
 *            times rescaled to [0, 2 pi]); INT32_MAX for an asset with fewer than two
 *            observations
 *   info     host: returns written, N = min_i N_i and the window (t0, T) = (t_min, t_max)
 *            to pass to mm_nufft1
 * All arrays are device memory; cap = n*D always suffices.  Synchronises `stream`.
 * Errors: MM_ERR_ARG; MM_ERR_DATA (a non-positive price, times not increasing within an
 * asset, a repeated time, or fewer than two distinct times overall); MM_ERR_WORKSPACE
 * (ws too small, or more than cap returns); MM_ERR_HIP. */
mm_status mm_matrix_to_csr(int64_t n, int32_t D, const double* P, const double* Tm, int64_t ld, int64_t* offsets,
                           double* t, void* dp, int32_t dp_is_fp64, int64_t cap, int32_t* nyq, void* ws,
                           size_t ws_bytes, mm_csr_info* info /* host */, void* stream);

/* Negative control: the zero-padded FFT method (its algorithm in the appendix)
 * puts every event on the nearest of Nstar equally spaced points of [t0, T)
 * (index l = round(Nstar (t - t0)/(T - t0)), l = Nstar wrapping to 0), then takes
 * an ordinary FFT.  This writes those moved times, out[i] = t0 + (T - t0) l/Nstar
 * (device float64[E]; out may equal t), so that mm_nufft1 on them gives exactly
 * what the zero-padded FFT computes (to tol).  On data already on such a grid (the
 * missing-data representation) nothing moves; under arrival-time asynchrony the
 * moves bias the estimate.  Asynchronous on `stream`.  Errors: MM_ERR_ARG, MM_ERR_HIP. */
mm_status mm_snap_times(int64_t E, const double* t, double t0, double T, int64_t Nstar, double* out, void* stream);

/* Human-readable text of a status (static storage). */
const char* mm_status_string(mm_status s);

/* Per-kernel timing: when enabled, every kernel the library launches is
 * bracketed by HIP events on its stream; mm_profile_read synchronises those
 * events and returns the summed duration and launch count of the kernels whose
 * name equals `kernel_name` (host string: the launched kernel's own name, e.g.
 * "k_spread_poly", "k_fft_rows_ab", "k_syrk_mfma256"), NULL meaning all.  Launches
 * inside a graph capture are not timed. */
mm_status mm_profile_enable(int32_t on);
mm_status mm_profile_read(const char* kernel_name, double* total_ms /* host */, int64_t* launches /* host */);
mm_status mm_profile_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* MM_H_ */
