// C ABI entry points (include/mm.h): argument checks on the host, plan and
// workspace carving, then asynchronous launches on the caller's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mm_internal.h"

namespace mm {

// ------------------------------------------------------------------------- profiling
namespace {
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_free;
std::map<std::string, std::pair<double, int64_t>> g_prof_total;
std::map<std::string, hipEvent_t> g_prof_open;

hipEvent_t take_event()
{
    if (!g_prof_free.empty()) {
        hipEvent_t e = g_prof_free.back();
        g_prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

thread_local bool g_prof_suspended = false;

void prof_begin(const char* name, hipStream_t st)
{
    if (!g_prof_on || g_prof_suspended) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e = take_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    g_prof_open[name] = e;
}

void prof_end(const char* name, hipStream_t st)
{
    if (!g_prof_on || g_prof_suspended) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    auto it = g_prof_open.find(name);
    if (it == g_prof_open.end()) return;
    hipEvent_t e = take_event();
    if (!e) return;
    (void)hipEventRecord(e, st);
    g_prof_pending.push_back({name, it->second, e});
    g_prof_open.erase(it);
}

static void prof_drain()
{
    for (auto& r : g_prof_pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(r.b);
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        auto& tot = g_prof_total[r.name];
        tot.first += ms;
        tot.second += 1;
        g_prof_free.push_back(r.a);
        g_prof_free.push_back(r.b);
    }
    g_prof_pending.clear();
}

}  // namespace mm

using namespace mm;

static mm_status hip_status(hipError_t e) { return e == hipSuccess ? MM_OK : MM_ERR_HIP; }

// Tables, then the NUFFT of all S series (host checks already done).
static hipError_t enqueue_nufft(const Plan& p, const NufftWs& w, char* wsb, int32_t S, const int64_t* offsets,
                                const double* t, const void* dp, int32_t dp_is_fp64, double t0, double T,
                                void* coef, int64_t ldc, hipStream_t st, const SplitOut* so = nullptr)
{
    if (p.prec == MM_MIXED) {
        // the tile ranges of every series come from the set-up launch when its
        // grids are resident at once (the fused kernel: one whole-grid tile each)
        const bool fz = use_fused(p, S);
        if (fz && so) return hipErrorInvalidValue;
        const bool one_pass = fz || S <= w.S_grid;
        const RangeReq rr{offsets, t, 0, S, fz ? 1 : (p.Mr + kRangeCells - 1) / kRangeCells,
                          fz ? kFusedMaxCells : kRangeCells, t0, T, (int64_t*)(wsb + w.ranges)};
        hipError_t e = launch_prep(p, w, wsb, st, one_pass ? &rr : nullptr, so);
        if (e != hipSuccess) return e;
        if (fz) return launch_nufft_fused(p, w, wsb, S, t, dp, dp_is_fp64, t0, T, coef, ldc, st);
        return launch_nufft_tiled(p, w, wsb, 0, S, offsets, t, dp, dp_is_fp64, t0, T, coef, ldc, st, so, one_pass);
    }
    hipError_t e = launch_prep(p, w, wsb, st);
    if (e != hipSuccess) return e;
    if (so) return hipErrorInvalidValue;
    // plain form: one launch chain per series, grid buffer reused in stream order
    for (int32_t sidx = 0; sidx < S && e == hipSuccess; ++sidx)
        e = launch_nufft_tiled(p, w, wsb, sidx, 1, offsets, t, dp, dp_is_fp64, t0, T, coef, ldc, st);
    return e;
}

static int small_d_limit(int32_t D) { return (int64_t)D * (D + 1) / 2 <= 1024; }

// The contraction for every cutoff, then the correlation (host checks already done).
static hipError_t enqueue_cov(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ns, int32_t nN,
                              int32_t Nmax, mm_basis basis, mm_prec prec, void* cov, void* corr, char* ws,
                              hipStream_t st, bool operands_ready = false, SyrkChoice sc = {})
{
    hipError_t e = hipSuccess;
    const size_t es = prec == MM_MIXED ? 4 : 8;
    if (small_d_limit(D)) {
        Cutoffs cut;
        cut.n = nN;
        for (int q = 0; q < nN; ++q) cut.N[q] = Ns[q];
        e = launch_cov_small(prec, G, D, coef, ldc, Nmax, cut, basis, cov, st, corr);
        return e;   // the correlations come from the same launch
    } else {
        // several cutoffs on the MFMA path: one pass over k where that costs less
        bool done = false;
        if (prec == MM_MIXED && nN >= 2 && !operands_ready) {
            e = launch_cov_mfma_sweep(G, D, coef, ldc, Ns, nN, basis, cov, ws, st, sc);
            done = e == hipSuccess;
            if (e == hipErrorNotSupported) e = hipSuccess;
        }
        for (int q = 0; !done && q < nN && e == hipSuccess; ++q) {
            char* cq = (char*)cov + (size_t)q * G * D * D * es;
            if (prec == MM_MIXED)
                e = launch_cov_mfma(G, D, coef, ldc, Ns[q], basis, cq, ws, st, operands_ready, sc);
            else
                e = launch_cov_fp64(G, D, coef, ldc, Ns[q], basis, cq, st);
        }
    }
    if (e == hipSuccess && corr) e = launch_corr(prec, (int64_t)nN * G, D, cov, corr, st);
    return e;
}

extern "C" {

const char* mm_status_string(mm_status s)
{
    switch (s) {
        case MM_OK: return "ok";
        case MM_ERR_ARG: return "invalid argument";
        case MM_ERR_DATA: return "invalid event data (unsorted, outside [t0,T] or non-finite)";
        case MM_ERR_TOL: return "tolerance outside the supported range for this precision";
        case MM_ERR_WORKSPACE: return "workspace too small";
        case MM_ERR_HIP: return "HIP runtime error";
        case MM_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

mm_status mm_plan_query(int32_t N, mm_kernel kernel, double tol, mm_prec prec, const mm_tuning* tune,
                        mm_plan_info* out)
{
    if (!out) return MM_ERR_ARG;
    Plan p;
    mm_status s = make_plan(N, kernel, tol, prec, tune, &p);
    if (s != MM_OK) return s;
    out->N = p.N;
    out->width = p.kp.w;
    out->msp = p.msp;
    out->Mr = p.Mr;
    out->L1 = p.L1;
    out->L2 = p.L2;
    out->fused = p.fused;
    out->tile = p.tile;
    out->sigma = p.sigma;
    out->beta = kernel == MM_ES ? p.kp.es_beta : (kernel == MM_GAUSSIAN ? p.kp.g_lambda : p.kp.kb_b);
    out->tol = p.tol;
    out->est_err = p.est_err;
    return MM_OK;
}

mm_status mm_nufft1_workspace_size(int32_t S, int32_t N, mm_kernel kernel, double tol, mm_prec prec,
                                   const mm_tuning* tune, size_t* bytes)
{
    if (!bytes || S < 0) return MM_ERR_ARG;
    Plan p;
    mm_status s = make_plan(N, kernel, tol, prec, tune, &p);
    if (s != MM_OK) return s;
    *bytes = nufft_workspace(p, S).total;
    return MM_OK;
}

mm_status mm_nufft1(int32_t S, const int64_t* offsets, const double* t, const void* dp, int32_t dp_is_fp64,
                    double t0, double T, int32_t N, mm_kernel kernel, double tol, mm_prec prec,
                    const mm_tuning* tune, void* coef, int64_t ldc, void* ws, size_t ws_bytes, int32_t validate,
                    void* stream)
{
    if (S < 0 || (dp_is_fp64 != 0 && dp_is_fp64 != 1) || (validate != 0 && validate != 1)) return MM_ERR_ARG;
    if (!isfinite(t0) || !isfinite(T) || !(T > t0)) return MM_ERR_ARG;
    if (N < 1 || ldc < (int64_t)N + 1) return MM_ERR_ARG;
    if (S > 0 && (!offsets || !t || !dp || !coef)) return MM_ERR_ARG;
    if (S > 65535) return MM_ERR_UNSUPPORTED;
    Plan p;
    mm_status s = make_plan(N, kernel, tol, prec, tune, &p);
    if (s != MM_OK) return s;
    NufftWs w = nufft_workspace(p, S);
    if (S == 0) return MM_OK;
    if (!ws || ws_bytes < w.total) return MM_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return MM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    char* wsb = (char*)ws;
    if (validate) {
        int* flag = (int*)(wsb + w.flag);
        if (hipMemsetAsync(flag, 0, sizeof(int), st) != hipSuccess) return MM_ERR_HIP;
        hipError_t e = launch_validate(S, offsets, t, dp, dp_is_fp64, t0, T, flag, st);
        if (e != hipSuccess) return MM_ERR_HIP;
        int host_flag = 0;
        if (hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return MM_ERR_HIP;
        if (hipStreamSynchronize(st) != hipSuccess) return MM_ERR_HIP;
        if (host_flag) return MM_ERR_DATA;
    }
    return hip_status(enqueue_nufft(p, w, wsb, S, offsets, t, dp, dp_is_fp64, t0, T, coef, ldc, st));
}

mm_status mm_cov_workspace_size(int32_t G, int32_t D, int32_t Nmax, int32_t nN, mm_prec prec, const mm_tuning* tune,
                                size_t* bytes)
{
    if (!bytes || G < 1 || D < 1 || Nmax < 1 || nN < 1 || nN > kMaxCutoffs) return MM_ERR_ARG;
    if (prec != MM_PLAIN_FP64 && prec != MM_MIXED) return MM_ERR_ARG;
    if (!syrk_choice_ok(tune)) return MM_ERR_ARG;
    *bytes = (small_d_limit(D) || prec == MM_PLAIN_FP64) ? 0 : cov_mfma_workspace(G, D, Nmax, syrk_choice(tune), nN);
    return MM_OK;
}

mm_status mm_cov(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ns, int32_t nN, mm_basis basis,
                 mm_prec prec, const mm_tuning* tune, void* cov, void* corr, void* ws, size_t ws_bytes, void* stream)
{
    if (G < 1 || D < 1 || !coef || !cov || !Ns || nN < 1 || nN > kMaxCutoffs) return MM_ERR_ARG;
    if (!syrk_choice_ok(tune)) return MM_ERR_ARG;
    if (basis != MM_DIRICHLET && basis != MM_FEJER) return MM_ERR_ARG;
    if (prec != MM_PLAIN_FP64 && prec != MM_MIXED) return MM_ERR_ARG;
    if ((int64_t)G * D > 65535ll * 65535ll) return MM_ERR_UNSUPPORTED;
    int32_t Nmax = 0;
    for (int q = 0; q < nN; ++q) {
        if (Ns[q] < 1 || (int64_t)Ns[q] > ldc - 1) return MM_ERR_ARG;
        Nmax = std::max(Nmax, Ns[q]);
    }
    size_t need = 0;
    mm_cov_workspace_size(G, D, Nmax, nN, prec, tune, &need);
    if (need > 0 && (!ws || ws_bytes < need)) return MM_ERR_WORKSPACE;
    if (need > 0 && ((uintptr_t)ws & 255) != 0) return MM_ERR_ARG;
    if (small_d_limit(D) && G > 65535) return MM_ERR_UNSUPPORTED;
    return hip_status(enqueue_cov(G, D, coef, ldc, Ns, nN, Nmax, basis, prec, cov, corr, (char*)ws,
                                  (hipStream_t)stream, false, syrk_choice(tune)));
}

}  // extern "C"

// ------------------------------------------------------------------------------ both stages
namespace {
struct EstLayout {
    size_t coef, nufft, cov, total;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

EstLayout est_layout(const Plan& p, int32_t S, int32_t G, int32_t D, int32_t Nmax, int32_t nN, const mm_tuning* tune)
{
    EstLayout L;
    const size_t cs = p.prec == MM_MIXED ? 8 : 16;
    size_t cw = 0;
    // room for the operands of the split fused into the row pass (one group, one
    // cutoff): L1 ceil((N+1)/L1) columns
    const int32_t Ncov = (G == 1 && nN == 1 && p.prec == MM_MIXED && p.fft_ab)
                             ? std::max(Nmax, split_out_cols(Nmax, p.L1) - 1) : Nmax;
    mm_cov_workspace_size(G, D, Ncov, nN, (mm_prec)p.prec, tune, &cw);
    L.coef = 0;
    L.nufft = al256((size_t)S * (size_t)(Nmax + 1) * cs);
    L.cov = L.nufft + al256(nufft_workspace(p, S).total);
    L.total = L.cov + al256(cw);
    return L;
}

// Graphs recorded by mm_estimate, keyed by the bytes of every argument.
std::mutex g_graph_mu;
std::map<std::string, hipGraphExec_t> g_graphs;
std::vector<std::string> g_graph_order;
constexpr size_t kMaxGraphs = 64;

template <typename V>
void put(std::string& k, const V& v)
{
    k.append(reinterpret_cast<const char*>(&v), sizeof(v));
}
}  // namespace

extern "C" {

mm_status mm_estimate_workspace_size(int32_t G, int32_t D, const int32_t* Ns, int32_t nN, mm_kernel kernel,
                                     double tol, mm_prec prec, const mm_tuning* tune, size_t* bytes)
{
    if (!bytes || !Ns || G < 1 || D < 1 || nN < 1 || nN > kMaxCutoffs) return MM_ERR_ARG;
    int32_t Nmax = 0;
    for (int q = 0; q < nN; ++q) {
        if (Ns[q] < 1) return MM_ERR_ARG;
        Nmax = std::max(Nmax, Ns[q]);
    }
    if ((int64_t)G * D > 65535) return MM_ERR_UNSUPPORTED;
    Plan p;
    mm_status s = make_plan(Nmax, kernel, tol, prec, tune, &p);
    if (s != MM_OK) return s;
    if (!syrk_choice_ok(tune)) return MM_ERR_ARG;
    *bytes = est_layout(p, G * D, G, D, Nmax, nN, tune).total;
    return MM_OK;
}

mm_status mm_estimate(int32_t G, int32_t D, const int64_t* offsets, const double* t, const void* dp,
                      int32_t dp_is_fp64, double t0, double T, const int32_t* Ns, int32_t nN, mm_basis basis,
                      mm_kernel kernel, double tol, mm_prec prec, const mm_tuning* tune, void* coef, int64_t ldc,
                      void* cov, void* corr, void* ws, size_t ws_bytes, int32_t use_graph, void* stream)
{
    if (G < 1 || D < 1 || !offsets || !t || !dp || !cov || !Ns || nN < 1 || nN > kMaxCutoffs) return MM_ERR_ARG;
    if ((dp_is_fp64 != 0 && dp_is_fp64 != 1) || (use_graph != 0 && use_graph != 1)) return MM_ERR_ARG;
    if (!isfinite(t0) || !isfinite(T) || !(T > t0)) return MM_ERR_ARG;
    if (basis != MM_DIRICHLET && basis != MM_FEJER) return MM_ERR_ARG;
    if (use_graph && !stream) return MM_ERR_ARG;   // the legacy default stream cannot be captured
    if ((int64_t)G * D > 65535) return MM_ERR_UNSUPPORTED;
    int32_t Nmax = 0;
    for (int q = 0; q < nN; ++q) {
        if (Ns[q] < 1) return MM_ERR_ARG;
        Nmax = std::max(Nmax, Ns[q]);
    }
    if (coef && ldc < (int64_t)Nmax + 1) return MM_ERR_ARG;
    Plan p;
    mm_status s = make_plan(Nmax, kernel, tol, prec, tune, &p);
    if (s != MM_OK) return s;
    if (!syrk_choice_ok(tune)) return MM_ERR_ARG;
    const SyrkChoice sc = syrk_choice(tune);
    const int32_t S = G * D;
    const EstLayout L = est_layout(p, S, G, D, Nmax, nN, tune);
    if (!ws || ws_bytes < L.total) return MM_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return MM_ERR_ARG;
    char* wsb = (char*)ws;
    const bool coef_out = coef != nullptr;
    if (!coef) {
        coef = wsb + L.coef;
        ldc = (int64_t)Nmax + 1;
    }
    const NufftWs w = nufft_workspace(p, S);
    hipStream_t st = (hipStream_t)stream;
    // With no coefficient output, one group and one cutoff on the MFMA path, the
    // FFT's row pass writes the contraction's BF16 operands directly, one FFT row
    // per run of columns (SplitOut).
    const bool fuse = !coef_out && G == 1 && nN == 1 && prec == MM_MIXED && !use_fused(p, S) && p.fft_ab &&
                      !small_d_limit(D);
    const SplitOut so = fuse ? cov_mfma_split_out(D, Ns[0], p.L1, wsb + L.cov, sc) : SplitOut{};
    // the contraction then runs on its operands' L1 K2 columns (zero beyond N)
    const int32_t Nop = fuse ? split_out_cols(Ns[0], p.L1) - 1 : Nmax;
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        if (fuse) {
            e = launch_split_prologue(D, Ns[0], p.L1, basis, wsb + L.cov, st, sc);
            if (e != hipSuccess) return e;
        }
        e = enqueue_nufft(p, w, wsb + L.nufft, S, offsets, t, dp, dp_is_fp64, t0, T, coef, ldc, st,
                          fuse ? &so : nullptr);
        if (e != hipSuccess) return e;
        return enqueue_cov(G, D, coef, ldc, fuse ? &Nop : Ns, nN, fuse ? Nop : Nmax, basis, prec, cov, corr,
                           wsb + L.cov, st, fuse, sc);
    };
    if (!use_graph) return hip_status(enqueue());

    std::string key;
    const void* ptrs[] = {offsets, t, dp, coef, cov, corr, ws, stream};
    put(key, G); put(key, D); put(key, dp_is_fp64); put(key, t0); put(key, T); put(key, nN);
    key.append(reinterpret_cast<const char*>(Ns), sizeof(int32_t) * (size_t)nN);
    put(key, basis); put(key, kernel); put(key, tol); put(key, prec); put(key, ldc); put(key, ws_bytes);
    put(key, coef_out);
    put(key, ptrs);
    const mm_tuning tz = tune ? *tune : mm_tuning{0, 0.0, 0, 0, 0.0, 0, 0, 0, 0, 0.0};
    put(key, tz.width); put(key, tz.sigma); put(key, tz.tile); put(key, tz.fused); put(key, tz.es_beta_per_tap);
    put(key, tz.fft_generic); put(key, tz.spread_direct); put(key, tz.syrk_tile); put(key, tz.syrk_splits);
    put(key, tz.moment_density);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MM_ERR_HIP;
    put(key, dev);

    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return MM_ERR_HIP;
        hipError_t e;
        {
            ProfSuspend quiet;   // event records are left out of captures
            e = enqueue();
        }
        hipError_t ec = hipStreamEndCapture(st, &graph);
        if (e != hipSuccess || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return MM_ERR_HIP;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return MM_ERR_HIP;
        if (g_graphs.size() >= kMaxGraphs) {
            // the oldest graph may still run on its stream: wait for the device before freeing it
            if (hipDeviceSynchronize() != hipSuccess) return MM_ERR_HIP;
            (void)hipGraphExecDestroy(g_graphs[g_graph_order.front()]);
            g_graphs.erase(g_graph_order.front());
            g_graph_order.erase(g_graph_order.begin());
        }
        it = g_graphs.emplace(key, exec).first;
        g_graph_order.push_back(key);
    }
    return hip_status(hipGraphLaunch(it->second, st));
}

mm_status mm_graph_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    if (!g_graphs.empty() && hipDeviceSynchronize() != hipSuccess) return MM_ERR_HIP;
    for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
    g_graph_order.clear();
    return MM_OK;
}

mm_status mm_matrix_to_csr_workspace_size(int64_t n, int32_t D, size_t* bytes)
{
    if (!bytes || n < 1 || D < 1) return MM_ERR_ARG;
    *bytes = input_workspace(n, D).total;
    return MM_OK;
}

mm_status mm_matrix_to_csr(int64_t n, int32_t D, const double* P, const double* Tm, int64_t ld, int64_t* offsets,
                           double* t, void* dp, int32_t dp_is_fp64, int64_t cap, int32_t* nyq, void* ws,
                           size_t ws_bytes, mm_csr_info* info, void* stream)
{
    if (n < 1 || D < 1 || ld < n || !P || !Tm || !offsets || !nyq || !info || cap < 0) return MM_ERR_ARG;
    if ((cap > 0 && (!t || !dp)) || (dp_is_fp64 != 0 && dp_is_fp64 != 1)) return MM_ERR_ARG;
    if (D > 65535) return MM_ERR_UNSUPPORTED;
    const InputWs w = input_workspace(n, D);
    if (!ws || ws_bytes < w.total) return MM_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return MM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    char* wsb = (char*)ws;
    if (launch_input(n, D, P, Tm, ld, offsets, t, dp, dp_is_fp64, nyq, w, wsb, st) != hipSuccess) return MM_ERR_HIP;
    int64_t meta[6];
    if (hipMemcpyAsync(meta, wsb + w.meta, sizeof(meta), hipMemcpyDeviceToHost, st) != hipSuccess) return MM_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return MM_ERR_HIP;
    const int64_t E = meta[0];
    if ((int)meta[2] != 0) return MM_ERR_DATA;
    if (E > cap) return MM_ERR_WORKSPACE;
    if (launch_input_returns(D, E, offsets, t, dp, dp_is_fp64, nyq, w, wsb, st) != hipSuccess) return MM_ERR_HIP;
    if (hipMemcpyAsync(meta, wsb + w.meta, sizeof(meta), hipMemcpyDeviceToHost, st) != hipSuccess) return MM_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return MM_ERR_HIP;
    double window[2];
    memcpy(window, &meta[4], sizeof(window));
    int32_t N;
    memcpy(&N, &meta[3], sizeof(N));
    if ((int)meta[2] != 0 || !(window[1] > window[0])) return MM_ERR_DATA;
    info->E = E;
    info->N = N;
    info->t0 = window[0];
    info->T = window[1];
    return MM_OK;
}

// Distinct ascending cutoffs of Ni and each asset's slot among them.
static bool pairwise_cutoffs(int32_t D, const int32_t* Ni, std::vector<int32_t>& Ns, std::vector<int32_t>& slot)
{
    Ns.assign(Ni, Ni + D);
    std::sort(Ns.begin(), Ns.end());
    Ns.erase(std::unique(Ns.begin(), Ns.end()), Ns.end());
    if (Ns.empty() || Ns.front() < 1) return false;
    slot.resize(D);
    for (int i = 0; i < D; ++i) slot[i] = (int32_t)(std::lower_bound(Ns.begin(), Ns.end(), Ni[i]) - Ns.begin());
    return true;
}

// Small D: the estimate swept over the distinct cutoffs (D <= 45, so at most 45 of
// them) and each entry read from its pair's slice.  Otherwise one product over the
// rows in ascending-cutoff order, whatever the number of distinct cutoffs.
static bool pairwise_sweep(int32_t D) { return small_d_limit(D); }

static size_t pairwise_layout(int32_t G, int32_t D, int32_t Nmax, int32_t nq, mm_prec prec, size_t* sweep_off,
                              size_t* cov_off)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    if (!pairwise_sweep(D)) {
        // tables: perm, Nr, rank, slot (D each) and cutq (Nmax + 1), then the product's workspace
        *sweep_off = 0;
        *cov_off = al(4 * (4 * (size_t)D + (size_t)Nmax + 1));
        return *cov_off + cov_pair_workspace(prec, G, D, Nmax, nq);
    }
    const size_t es = prec == MM_MIXED ? 4 : 8;
    size_t cw = 0;
    mm_cov_workspace_size(G, D, Nmax, nq, prec, nullptr, &cw);
    *sweep_off = al(4 * (size_t)D);
    *cov_off = *sweep_off + al((size_t)nq * G * D * D * es);
    return *cov_off + al(cw);
}

mm_status mm_cov_pairwise_workspace_size(int32_t G, int32_t D, const int32_t* Ni, mm_prec prec, size_t* bytes)
{
    if (!bytes || !Ni || G < 1 || D < 1 || (prec != MM_PLAIN_FP64 && prec != MM_MIXED)) return MM_ERR_ARG;
    std::vector<int32_t> Ns, slot;
    if (!pairwise_cutoffs(D, Ni, Ns, slot)) return MM_ERR_ARG;
    size_t a, b;
    *bytes = pairwise_layout(G, D, Ns.back(), (int32_t)Ns.size(), prec, &a, &b);
    return MM_OK;
}

mm_status mm_cov_pairwise(int32_t G, int32_t D, const void* coef, int64_t ldc, const int32_t* Ni, mm_basis basis,
                          mm_prec prec, void* cov, void* corr, void* ws, size_t ws_bytes, void* stream)
{
    if (G < 1 || D < 1 || !coef || !cov || !Ni) return MM_ERR_ARG;
    if (basis != MM_DIRICHLET && basis != MM_FEJER) return MM_ERR_ARG;
    if (prec != MM_PLAIN_FP64 && prec != MM_MIXED) return MM_ERR_ARG;
    std::vector<int32_t> Ns, slot;
    if (!pairwise_cutoffs(D, Ni, Ns, slot)) return MM_ERR_ARG;
    const int32_t nq = (int32_t)Ns.size(), Nmax = Ns.back();
    if ((int64_t)Nmax > ldc - 1) return MM_ERR_ARG;
    if (pairwise_sweep(D) && G > 65535) return MM_ERR_UNSUPPORTED;
    if (!pairwise_sweep(D) && (D > 65535 || G > 65535)) return MM_ERR_UNSUPPORTED;
    size_t sweep_off, cov_off;
    const size_t need = pairwise_layout(G, D, Nmax, nq, prec, &sweep_off, &cov_off);
    if (!ws || ws_bytes < need) return MM_ERR_WORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return MM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    char* wsb = (char*)ws;
    hipError_t e;
    if (pairwise_sweep(D)) {
        if (hipMemcpyAsync(wsb, slot.data(), 4 * (size_t)D, hipMemcpyHostToDevice, st) != hipSuccess)
            return MM_ERR_HIP;
        e = enqueue_cov(G, D, coef, ldc, Ns.data(), nq, Nmax, basis, prec, wsb + sweep_off, nullptr, wsb + cov_off,
                        st);
        if (e == hipSuccess)
            e = launch_pairwise_select(prec, G, D, (const int32_t*)wsb, wsb + sweep_off, cov, corr, st);
    } else {
        // rows in ascending order of cutoff (stable), their cutoffs, ranks and slots,
        // and the slot of every k that is a cutoff
        std::vector<int32_t> tab(4 * (size_t)D + (size_t)Nmax + 1, -1);
        int32_t* perm = tab.data();
        int32_t* Nr = perm + D;
        int32_t* rank = Nr + D;
        int32_t* rslot = rank + D;
        int32_t* cutq = rslot + D;
        for (int i = 0; i < D; ++i) perm[i] = i;
        std::stable_sort(perm, perm + D, [&](int32_t a, int32_t b) { return Ni[a] < Ni[b]; });
        for (int r = 0; r < D; ++r) {
            Nr[r] = Ni[perm[r]];
            rank[perm[r]] = r;
            rslot[r] = slot[perm[r]];
        }
        for (int q = 0; q < nq; ++q) cutq[Ns[q]] = q;
        if (hipMemcpyAsync(wsb, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice, st) != hipSuccess)
            return MM_ERR_HIP;
        const int32_t* dt = (const int32_t*)wsb;
        const PairTables tb{dt, dt + D, dt + 2 * D, dt + 3 * D, dt + 4 * D};
        e = launch_cov_pair(prec, G, D, coef, ldc, Nmax, tb, nq, basis, cov, corr, wsb + cov_off, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host tables must outlive the copy
    return hip_status(e);
}

mm_status mm_snap_times(int64_t E, const double* t, double t0, double T, int64_t Nstar, double* out, void* stream)
{
    if (E < 0 || Nstar < 1 || !isfinite(t0) || !isfinite(T) || !(T > t0)) return MM_ERR_ARG;
    if (E > 0 && (!t || !out)) return MM_ERR_ARG;
    return hip_status(launch_snap(E, t, t0, T, Nstar, out, (hipStream_t)stream));
}

mm_status mm_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return MM_OK;
}

mm_status mm_profile_read(const char* name, double* total_ms, int64_t* launches)
{
    if (!total_ms || !launches) return MM_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    double ms = 0;
    int64_t n = 0;
    for (auto& kv : g_prof_total)
        if (!name || kv.first == name) {
            ms += kv.second.first;
            n += kv.second.second;
        }
    *total_ms = ms;
    *launches = n;
    return MM_OK;
}

mm_status mm_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    g_prof_total.clear();
    return MM_OK;
}

}  // extern "C"
