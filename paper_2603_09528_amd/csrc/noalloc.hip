// Allocation-free solve: tpt_solve with its workspace taken from a static
// device array instead of caller memory or a plan-owned allocation, for
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array lives in this code object, one copy per GPU the library runs on,
// held until the process ends.  In host code its name is only a host-side
// stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress and that address is what the solve receives.  Every
// call on one GPU uses the same array: calls that overlap on a GPU (other
// streams, other threads) race on it.  Nothing in it needs clearing between
// calls: each kernel of a solve writes its part of the workspace before any
// kernel reads it.
#include <mutex>

#include "internal.h"

namespace tpt {
namespace {

constexpr size_t STATIC_WS_BYTES = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_ws_mu;
void* g_ws_ptr[MAX_DEVICES] = {nullptr};

// Device address of this device's copy of the array (looked up on the first
// call on that device, with the device current).
int static_workspace(int device, void** ptr) {
    if (device < 0 || device >= MAX_DEVICES) return fail(TPT_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_ws_mu);
    if (!g_ws_ptr[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TPT_ERR_HIP, std::string("hipGetSymbolAddress of the static workspace: ") +
                                         hipGetErrorString(e));
        g_ws_ptr[device] = p;
    }
    *ptr = g_ws_ptr[device];
    return TPT_OK;
}

}  // namespace
}  // namespace tpt

using namespace tpt;

extern "C" {

size_t tpt_static_workspace_capacity(void) { return STATIC_WS_BYTES; }

int tpt_solve_noalloc(tpt_plan plan, const double* rhs, double* out, void* stream) {
    if (!plan) return fail(TPT_ERR_INVALID, "NULL plan");
    if (plan->host_only) return fail(TPT_ERR_INVALID, "host-only plan cannot solve");
    const size_t need = plan_workspace_bytes(plan);
    if (need > STATIC_WS_BYTES)
        return fail(TPT_ERR_WORKSPACE, "tpt_solve_noalloc: the plan needs " + std::to_string(need) +
                                           " bytes of workspace, above the static workspace of " +
                                           std::to_string(STATIC_WS_BYTES) + " bytes; use tpt_solve");
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) TPT_HIP(hipSetDevice(plan->device));
    void* ws = nullptr;
    int rc = static_workspace(plan->device, &ws);
    if (rc) return rc;
    return solve_one(plan, rhs, out, ws, STATIC_WS_BYTES, (hipStream_t)stream);
}

}  // extern "C"
