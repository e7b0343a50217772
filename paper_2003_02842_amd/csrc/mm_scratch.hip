// mm_estimate_noalloc: mm_estimate for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  Its workspace is
// a file-scope device array of fixed size instead of a caller's buffer.
//
// Each GPU the library runs on holds its own copy of the array until the process
// ends.  In host code the array's name is only a stand-in for the device symbol,
// so its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and that pointer is what the launches receive.
// Calls on one GPU share its array: two calls that overlap in time on one GPU
// race, and each call leaves its contents behind (no kernel of mm_estimate reads
// workspace it has not written in the same call, so nothing is cleared).
#include <hip/hip_runtime.h>

#include <mutex>

#include "mm_internal.h"

namespace mm {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // mm.h: MM_SCRATCH_BYTES
static_assert(kScratchBytes == MM_SCRATCH_BYTES, "scratch size and its declaration differ");

__device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each device, once looked up

// The array's device address on the current device (looked up on the first call
// made with that device current).
hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidValue;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

}  // namespace mm

using namespace mm;

extern "C" mm_status mm_estimate_noalloc(int32_t G, int32_t D, const int64_t* offsets, const double* t,
                                         const void* dp, int32_t dp_is_fp64, double t0, double T, const int32_t* Ns,
                                         int32_t nN, mm_basis basis, mm_kernel kernel, double tol, mm_prec prec,
                                         const mm_tuning* tune, void* coef, int64_t ldc, void* cov, void* corr,
                                         void* stream)
{
    // the host checks of mm_estimate, so that bad arguments fail the same way
    if (G < 1 || D < 1 || !offsets || !t || !dp || !cov || !Ns || nN < 1 || nN > kMaxCutoffs) return MM_ERR_ARG;
    size_t need = 0;
    const mm_status s = mm_estimate_workspace_size(G, D, Ns, nN, kernel, tol, prec, tune, &need);
    if (s != MM_OK) return s;
    if (need > kScratchBytes) return MM_ERR_WORKSPACE;   // the problem does not fit the fixed scratch
    void* ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return MM_ERR_HIP;
    // no per-kernel timing inside: its events would be created on demand
    ProfSuspend quiet;
    return mm_estimate(G, D, offsets, t, dp, dp_is_fp64, t0, T, Ns, nN, basis, kernel, tol, prec, tune, coef, ldc,
                       cov, corr, ws, kScratchBytes, 0, stream);
}
