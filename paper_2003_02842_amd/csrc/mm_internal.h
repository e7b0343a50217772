// Internal declarations shared by the host runtime (mm_api.cpp, mm_plan.cpp)
// and the gfx950 kernels (mm_nufft.hip, mm_cov.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

#include "mm.h"

namespace mm {

constexpr int kMaxStages = 12;     // radix stages of one in-LDS sub-FFT
constexpr int kMaxSub = 2048;      // longest in-LDS sub-FFT
constexpr int kMaxTaps = 40;       // spreading taps per event
constexpr int kMaxCutoffs = 128;   // cutoffs per mm_cov call
constexpr int kGLNodes = 64;       // positive nodes of the 128-point Gauss-Legendre rule
constexpr int kFusedMaxCells = 8192;          // largest grid of the fused single-workgroup NUFFT
constexpr size_t kFusedMaxLds = 80 * 1024;    // its LDS budget (two workgroups per CU)
constexpr double kMomDensity = 3.0;         // events per cell from which a tile spreads from moments
constexpr int kRangeCells = 1024;           // cells per event-range sub-tile (spreading tiles are 1-4 of them)
constexpr int kFusedMinSeries = 64;           // series from which the planner's "auto" takes it

// Exact unsigned division a / d for a < 2^22, d < 2^20: (a * M) >> 42, M = ceil(2^42/d).
struct FastDiv {
    uint64_t M;
    uint32_t d;
};

// One in-place decimation-in-frequency FFT of length n held in LDS.
struct FFTDesc {
    int n;
    int ns;                   // number of radix stages
    int r[kMaxStages];        // radix of stage s (2, 3, 4 or 5)
    int m[kMaxStages];        // span / radix of stage s
    int tws[kMaxStages];      // twiddle-table stride n / span of stage s
    FastDiv dm[kMaxStages];   // division by m[s]
    FastDiv dnr[kMaxStages];  // division by n / r[s]
    // LDS passes: each applies one stage (p2 = 1) or two consecutive stages
    // (radix p1 then p2) to p1*p2 values a thread keeps in registers.
    int np;
    int p1[kMaxStages], p2[kMaxStages];
    int pm1[kMaxStages], pm2[kMaxStages], plen[kMaxStages];
    int pts1[kMaxStages], pts2[kMaxStages];
    FastDiv pdtask[kMaxStages];   // division by n / (p1 p2), tasks per transform
    FastDiv pdm2[kMaxStages];     // division by tasks per block
};

// Averaging-kernel parameters in grid units (x = cell distance).
struct KernParams {
    int kind;        // MM_GAUSSIAN / MM_KAISER_BESSEL / MM_ES
    int w;           // taps per event
    double hw;       // w / 2: first tap sits at floor(g - hw) + 1
    // ES: exp(beta (sqrt(1 - (x/hw)^2) - 1))
    double es_beta, es_inv_hw;
    // Gaussian: exp(-t1 x^2), t1 = pi / lambda; FGG tables e3[k] = exp(-t1 k^2)
    double g_t1, g_lambda;
    int g_msp;
    double g_e3[kMaxTaps / 2 + 1];
    // Kaiser-Bessel: inv_norm * sinh(b s)/s, s = sqrt(m^2 - x^2) (sin branch outside)
    double kb_b, kb_m, kb_inv_norm;
};

// Per-tap polynomials of the averaging kernel for the FP32 spreading path:
// tap j of an event with cell fraction f has value sum_k c[j][k] s^k, s = f - 1/2
// (the kernel at x = j + 1/2 - s - hw; Chebyshev interpolation, monomial form).
// The kernel is even, so tap w-1-j is the same polynomial at -s; rows j < ceil(w/2)
// are filled.
constexpr int kMaxPolyTaps = 16;
constexpr int kMaxPolyDeg = 12;
struct PolyParams {
    int deg;
    float c[kMaxPolyTaps][kMaxPolyDeg + 1];
};
// Degree of the per-tap polynomials for a given width.  With FP32 coefficients
// the fits of the ES, Kaiser-Bessel and Gaussian shapes at sigma = 1.55..2.5
// stop improving at degree 8 (largest deviation 1e-8..4.4e-8 for widths 8-16);
// narrower kernels, used at looser tolerances, take fewer terms.  The planner
// checks every fit and otherwise evaluates the kernel formula.
__host__ __device__ constexpr int poly_degree_for_width(int w)
{
    return w <= 2 ? 4 : (w <= 3 ? 5 : (w <= 5 ? 6 : (w <= 6 ? 7 : 8)));
}
// Widths of degree 8 also run at degree 7 where that fit leaves the error
// estimate within tol (the planner's choice; the large-grid spreading kernels
// have instances of both, the others evaluate degree 8 with a zero top term).
constexpr int kPolyDegTop = 8;
constexpr int kPolyDegLow = 7;

struct Plan {
    int prec;            // mm_prec
    int kernel;          // mm_kernel
    int N, M;            // cutoff and M = 2N + 1
    double tol, sigma;
    int msp;             // spreading half-width M_sp of the paper's tolerance rule
    int wmsp;            // half-width parameter of the kernel actually used
    double est_err;      // a-priori worst-case relative coefficient error
    int Mr, L, L1, L2;   // real grid length, complex length Mr/2 = L1 * L2
    int L2p;             // row pitch (complex) of the L1 x L2 grid view: L2 rounded up to 128 bytes
    KernParams kp;
    FFTDesc F1, F2;
    int CB;              // columns per block of the column pass
    int R;               // row pairs per block of the row pass
    // two-pass sub-transforms with one LDS exchange (mm_fft.hip): L1 = A1 B1, L2 = A2 B2
    int fft_ab;          // 1: both sub-lengths split into codelet sizes <= 32
    int A1, B1, A2, B2;
    int CC;              // columns per block of the column pass
    int RR;              // row pairs per block of the row pass
    int tw_lo_bits;      // split twiddle tables W^m = lo[m mod 2^bits] hi[m >> bits]
    int tw_hi_L, tw_hi_M;
    int poly;            // 1: FP32 spreading from per-tap polynomials (mm_nufft.hip, k_spread_poly)
    double poly_err;     // largest deviation of the polynomials from the kernel (FP64 evaluation)
    PolyParams pp;
    int tile;            // cells per spreading tile: 1024, 2048 or 4096 (256 threads x 4, 8, 16 cells)
    double mom_density;  // > 0: tiles with at least this many events per cell spread from per-cell
                         // moments (k_spread_mom); 0: all by k_spread_poly
    int fused;           // 1: the fused single-workgroup NUFFT can run this plan (mm_fused.hip)
    int fused_min_series;   // ... and runs it for calls with at least this many series
};

// Whether a call on S series takes the fused single-workgroup NUFFT.
inline bool use_fused(const Plan& p, int32_t S) { return p.fused && S >= p.fused_min_series; }

// Plan construction (host only, no device calls).  Returns MM_OK or an error.
mm_status make_plan(int32_t N, mm_kernel kernel, double tol, mm_prec prec, const mm_tuning* tune, Plan* p);
uint64_t smooth_even_at_least(uint64_t n);
FastDiv make_fastdiv(uint32_t d);
void gauss_legendre_pos(int n_pos, double* x, double* w);   // nodes/weights on (0,1] of a 2n_pos rule on [-1,1]
// What the planner checks against the kernels' LDS (layouts in mm_layout.h): the
// codelet split n = A x B of a two-pass FFT and the LDS of its column and row
// passes; whether the fused small-grid NUFFT can run a plan, and its LDS.
bool fft_ab_split(int n, int max_codelet, int* A, int* B);
size_t fft_ab_lds_cols(const Plan& p);
size_t fft_ab_lds_rows(const Plan& p);
bool fused_fits(const Plan& p);
size_t fused_lds_bytes(const Plan& p);

// Workspace layout of one mm_nufft1 call.
struct NufftWs {
    size_t tw1, tw2, twL, twM, rev1, pos2, dfac, flag, ranges, grid, total;
    size_t tLlo, tLhi, tMlo, tMhi;   // split twiddle tables of the two-pass FFT
    int S_grid;   // series whose grids are resident at once
};
NufftWs nufft_workspace(const Plan& p, int32_t S);

// Launchers (mm_nufft.hip).  All asynchronous on `st`.
// Tile event ranges for the set-up launch to compute as well: the series
// [s_begin, s_begin + s_count) over tiles of tc cells, into `ranges`.
struct RangeReq {
    const int64_t* offsets;
    const double* t;
    int32_t s_begin, s_count;
    int tiles, tc;
    double t0, T;
    int64_t* ranges;
};
struct SplitOut;
// Deconvolution factors and FFT tables (one launch with the two-pass FFT, which
// also takes the tile ranges of rr, and writes the fused split's column factors
// so->fac from its scale table), before the spreading.
hipError_t launch_prep(const Plan& p, const NufftWs& w, char* ws, hipStream_t st, const RangeReq* rr = nullptr,
                       const SplitOut* so = nullptr);
hipError_t launch_validate(int32_t S, const int64_t* offsets, const double* t, const void* dp, int dp_fp64,
                           double t0, double T, int* flag, hipStream_t st);
// Destination of the split fused into the FFT's row pass: X = s_k c_k as BF16 hi
// and lo parts (a uint32 pair (Re, Im)) in the MFMA contraction's operand rows
// (row = series) instead of the coefficients c_k.  Coefficient k = k1 + L1 k2 sits
// at column k1 K2 + k2, K2 = ceil((N + 1) / L1): the row pass transforms one FFT row
// (one k1) at a time, so each of its rows leaves as one contiguous run, and the
// contraction's sum over k does not depend on the order of the columns.  Columns
// whose k exceeds N hold zero.
struct SplitOut {
    uint32_t* hi;
    uint32_t* lo;
    int64_t kp2;           // pairs per operand row (Kp / 2), at least L1 K2
    int32_t k2n;           // K2
    const float* scale;    // s_k by k, zero beyond N (written by the prologue)
    float* fac;            // by column: s_k d_k / 2 (d_k the deconvolution factor), zero where k > N
};
// Columns of the fused split's operands for cutoff N and FFT row count L1: L1 K2.
int32_t split_out_cols(int32_t N, int32_t L1);


hipError_t launch_nufft_tiled(const Plan& p, const NufftWs& w, char* ws, int32_t s_begin, int32_t s_count,
                              const int64_t* offsets, const double* t, const void* dp, int dp_fp64,
                              double t0, double T, void* coef, int64_t ldc, hipStream_t st,
                              const SplitOut* so = nullptr, bool ranges_ready = false);
hipError_t launch_spread_poly(const Plan& p, int s_count, const double* t, const void* dp, int dp_fp64, double t0,
                              double t_end, const int64_t* ranges, int nsub, float* grid, int64_t grid_stride,
                              hipStream_t st);
// Fused small-grid NUFFT (mm_fused.hip): one workgroup per series from events to
// coefficients, on the ranges of one whole-grid tile per series (launch_prep).
hipError_t launch_nufft_fused(const Plan& p, const NufftWs& w, char* ws, int32_t S, const double* t, const void* dp,
                              int dp_fp64, double t0, double T, void* coef, int64_t ldc, hipStream_t st);
// Event ranges of every (series, tile of tc cells) (k_tile_ranges).
hipError_t launch_tile_ranges(const Plan& p, const int64_t* offsets, const double* t, int32_t s_begin,
                              int32_t s_count, int tiles, int tc, double t0, double T, int64_t* ranges,
                              hipStream_t st);

// Two-pass grid FFT with one LDS exchange per pass (mm_fft.hip).
hipError_t launch_fft_ab_tables(const Plan& p, const NufftWs& w, char* ws, hipStream_t st);
hipError_t launch_fft_ab(const Plan& p, const NufftWs& w, char* ws, int32_t s_begin, int32_t s_count, void* grid,
                         int64_t gstride, void* coef, int64_t ldc, hipStream_t st, const SplitOut* so = nullptr);

// Paper-form input (mm_input.hip): price/time matrices to CSR returns.
struct InputWs {
    size_t cnt, tmin, tmax, mindt, voff, meta, tv, lv, total;
};
InputWs input_workspace(int64_t n, int32_t D);
hipError_t launch_input(int64_t n, int32_t D, const double* P, const double* Tm, int64_t ld, int64_t* offsets,
                        double* t, void* dp, int dp_fp64, int32_t* nyq, const InputWs& w, char* ws, hipStream_t st);
hipError_t launch_snap(int64_t E, const double* t, double t0, double T, int64_t Nstar, double* out, hipStream_t st);
hipError_t launch_input_returns(int32_t D, int64_t E, int64_t* offsets, double* t, void* dp, int dp_fp64,
                                int32_t* nyq, const InputWs& w, char* ws, hipStream_t st);

// Shape of the MFMA contraction requested by a caller's tuning (mm_tuning.syrk_tile,
// syrk_splits); 0 leaves the choice to the built-in model.
struct SyrkChoice {
    int tile = 0;
    int splits = 0;
};
inline SyrkChoice syrk_choice(const mm_tuning* t) { return t ? SyrkChoice{t->syrk_tile, t->syrk_splits} : SyrkChoice{}; }
inline bool syrk_choice_ok(const mm_tuning* t)
{
    return !t || ((t->syrk_tile == 0 || t->syrk_tile == 128 || t->syrk_tile == 256) && t->syrk_splits >= 0);
}

// Contraction launchers (mm_cov.hip).
struct Cutoffs {
    int n;
    int N[kMaxCutoffs];
};
// (with corr, the correlations too, in the same launch)
hipError_t launch_cov_small(int prec, int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t Nmax,
                            const Cutoffs& cut, int basis, void* cov, hipStream_t st, void* corr = nullptr);
hipError_t launch_corr(int prec, int64_t mats, int32_t D, const void* cov, void* corr, hipStream_t st);
// (with nN >= 2, also enough for the one-pass sweep of nN cutoffs)
size_t cov_mfma_workspace(int32_t G, int32_t D, int32_t Nmax, SyrkChoice sc = {}, int32_t nN = 1);
// The MFMA contraction of nN >= 2 cutoffs in one pass over k (segment Gram
// matrices, summed in k order): hipErrorNotSupported where the cutoffs exceed its
// tables or where separate products per cutoff cost less (the caller runs those).
hipError_t launch_cov_mfma_sweep(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ns, int32_t nN,
                                 int basis, void* cov, char* ws, hipStream_t st, SyrkChoice sc = {});
hipError_t launch_pairwise_select(int prec, int32_t G, int32_t D, const int32_t* qidx, const void* sweep, void* cov,
                                  void* corr, hipStream_t st);
// operands_ready: the split operands were written by the NUFFT's row pass
// (launch_split_prologue, then SplitOut), so the scale and split steps are skipped.
hipError_t launch_cov_mfma(int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t N, int basis,
                           void* cov, char* ws, hipStream_t st, bool operands_ready = false, SyrkChoice sc = {});
// The fused split for one group and one cutoff N of the MFMA contraction (the
// NUFFT's FFT having L1 rows): the operand pointers in its workspace, which is
// that of cutoff split_out_cols(N, L1) - 1, and a prologue that writes the scale
// table s_k and zeroes the operands' padding (rows D..Dp-1, columns from L1 K2 on).
// The NUFFT's set-up launch then fills SplitOut::fac.
SplitOut cov_mfma_split_out(int32_t D, int32_t N, int32_t L1, char* ws, SyrkChoice sc = {});
hipError_t launch_split_prologue(int32_t D, int32_t N, int32_t L1, int basis, char* ws, hipStream_t st,
                                 SyrkChoice sc = {});
hipError_t launch_cov_fp64(int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t N, int basis,
                           void* cov, hipStream_t st);
// The one-pass per-pair-cutoff product (mm_cov_pairwise beyond the small-D path):
// device tables of the rows in ascending-cutoff order.
struct PairTables {
    const int32_t* perm;   // [D] series of sorted row r
    const int32_t* Nr;     // [D] cutoff of sorted row r
    const int32_t* rank;   // [D] sorted row of series a
    const int32_t* slot;   // [D] index of Nr[r] among the distinct cutoffs
    const int32_t* cutq;   // [Nmax + 1] index of k among the distinct cutoffs, -1 if none
};
size_t cov_pair_workspace(int prec, int32_t G, int32_t D, int32_t Nmax, int32_t nq);
hipError_t launch_cov_pair(int prec, int32_t G, int32_t D, const void* coef, int64_t ldc, int32_t Nmax,
                           const PairTables& tb, int32_t nq, int basis, void* cov, void* corr, char* ws,
                           hipStream_t st);

// Optional per-kernel timing with HIP events on the launch stream.
void prof_begin(const char* name, hipStream_t st);
void prof_end(const char* name, hipStream_t st);
// Set on a thread while its launches must not be timed (a graph capture, or the
// allocation-free entry point, whose events would be created on demand).
extern thread_local bool g_prof_suspended;
struct ProfSuspend {
    bool prev;
    ProfSuspend() : prev(g_prof_suspended) { g_prof_suspended = true; }
    ~ProfSuspend() { g_prof_suspended = prev; }
};

}  // namespace mm
