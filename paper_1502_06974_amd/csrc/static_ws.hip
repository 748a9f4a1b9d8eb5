// wcal_solve_static: the batched solve with its workspace in a static device array, for
// callers that cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// `scratch` is a file-scope __device__ array: every GPU the library runs on holds its own copy
// (WCAL_STATIC_WORKSPACE_BYTES) from the module's load until the process ends.  In host code
// the name stands for a host-side shadow, not a device address, so the device address is
// looked up once per device (hipGetSymbolAddress, with that device current) and only that
// address is handed to the kernels.  The solve initialises every part of its workspace that
// it reads, so what a previous call left there does not matter; calls that overlap on one GPU
// (two streams, two host threads) share the array and race.
#include <mutex>
#include <string>

#include "wcal_internal.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[WCAL_STATIC_WORKSPACE_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first call).
int scratch_of(int device, void** out) {
    if (device < 0 || device >= kMaxDevices)
        return wcal_error(WCAL_EINVAL, "device index " + std::to_string(device) + " beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        if (hipSetDevice(device) != hipSuccess) return wcal_error(WCAL_EHIP, "hipSetDevice failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return wcal_error(WCAL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return WCAL_OK;
}

}  // namespace

extern "C" int wcal_solve_static(wcal_plan* plan, const wcal_c64* data, const wcal_c64* model, const uint8_t* flags,
                                 wcal_c64* gains, wcal_c64* residual, int32_t* n_iter, uint32_t* status, double* chi2,
                                 void* stream) {
    if (!plan) return wcal_error(WCAL_EINVAL, "plan is NULL");
    if (plan->ws_bytes > WCAL_STATIC_WORKSPACE_BYTES)
        return wcal_error(WCAL_ENOMEM, "the plan needs a workspace of " + std::to_string(plan->ws_bytes) +
                                           " bytes, the static one holds " +
                                           std::to_string((size_t)WCAL_STATIC_WORKSPACE_BYTES) +
                                           " (use wcal_solve with a caller-owned workspace)");
    if (plan->prof) return wcal_error(WCAL_EINVAL, "profiling creates HIP events; disable it for wcal_solve_static");
    void* ws = nullptr;
    if (int rc = scratch_of(plan->device, &ws)) return rc;
    return wcal_solve(plan, data, model, flags, gains, residual, n_iter, status, chi2, ws,
                      (size_t)WCAL_STATIC_WORKSPACE_BYTES, stream);
}
