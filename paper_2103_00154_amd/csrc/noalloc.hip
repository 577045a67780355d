// noalloc.hip - dsg_peel_async_noalloc: dsg_peel_async for callers that
// cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  The workspace is a
// static device array of kScratchBytes, one per GPU the library runs on,
// held until the process ends.
//
// Host code never passes the array's name to a kernel (on the host it is
// only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current on
// the first call there, and kept per device.

#include <hip/hip_runtime.h>

#include <mutex>

#include "dsg.h"
#include "host.h"

namespace {

// 256 MiB: the peel workspace of graphs up to about n = 2^20 vertices with
// m = 16 M edges (R-MAT scale 20); dsg_workspace_bytes(n, m) must fit.
constexpr size_t kScratchBytes = size_t(256) << 20;

__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int32_t dsg_peel_async_noalloc(const dsg_csr* g, int64_t n, int64_t m, int64_t eps_num,
                               int64_t eps_den, int32_t* best_ids, int32_t* removed_at,
                               dsg_batch_result* result, const dsg_launch* launch,
                               void* stream) {
    if (!g || !result) return DSG_EINVAL;
    const int32_t rc = dsg::check_sizes(n, m, eps_num, eps_den);
    if (rc != DSG_OK) return rc;
    const size_t need = dsg_workspace_bytes(n, m);
    if (need == 0 || need > kScratchBytes) return DSG_EINVAL;  // graph too large
    void* ws = nullptr;
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return dsg::map_hip(e);
    return dsg::peel_async(g, n, m, eps_num, eps_den, best_ids, removed_at, result, launch, ws,
                           kScratchBytes, stream);
}

}  // extern "C"
