// validate.hip - device check of the CSR input contract of include/dsg.h
// (dsg_validate_csr).  Two kernels: the first reads only row_ptr; the second
// reads rows only once row_ptr is known to describe ranges inside col_idx,
// so no access can leave the caller's buffers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "dsg.h"

namespace dsg {
namespace {

// rule numbers (smallest violated one is reported)
enum : int32_t { kRuleFirst = 1, kRuleMono = 2, kRuleLast = 3, kRuleRange = 4, kRuleLoop = 5,
                 kRuleOrder = 6, kRuleReverse = 7, kRuleNone = 1000 };

__global__ __launch_bounds__(kBlock) void k_check_rowptr(const int32_t* __restrict__ rp,
                                                         int64_t n, int64_t m,
                                                         int32_t* __restrict__ rule) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
        if (rp[v + 1] < rp[v]) atomicMin(rule, (int32_t)kRuleMono);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (rp[0] != 0) atomicMin(rule, (int32_t)kRuleFirst);
        if ((int64_t)rp[n] != 2 * m) atomicMin(rule, (int32_t)kRuleLast);
    }
}

// One wave per row; lanes stride over the row's entries.
__global__ __launch_bounds__(kBlock) void k_check_rows(const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, int64_t n,
                                                       int32_t* __restrict__ rule) {
    const int64_t waves = (int64_t)gridDim.x * kWaves;
    const int lane = lane_id();
    int32_t found = kRuleNone;
    for (int64_t v = (int64_t)blockIdx.x * kWaves + wave_id(); v < n; v += waves) {
        const int64_t lo = rp[v], hi = rp[v + 1];
        for (int64_t e = lo + lane; e < hi; e += 64) {
            const int32_t u = ci[e];
            if (u < 0 || (int64_t)u >= n) {
                found = min(found, (int32_t)kRuleRange);
                continue;
            }
            if ((int64_t)u == v) found = min(found, (int32_t)kRuleLoop);
            if (e > lo && ci[e - 1] >= u) found = min(found, (int32_t)kRuleOrder);
            // reverse entry v in row u (binary search; rows may be unsorted,
            // which rule 6 reports)
            int64_t a = rp[u], b = rp[u + 1];
            bool ok = false;
            while (a < b) {
                const int64_t mid = a + (b - a) / 2;
                const int32_t x = ci[mid];
                if ((int64_t)x == v) {
                    ok = true;
                    break;
                }
                if ((int64_t)x < v) a = mid + 1;
                else b = mid;
            }
            if (!ok) found = min(found, (int32_t)kRuleReverse);
        }
    }
    if (found != kRuleNone) atomicMin(rule, found);
}

}  // namespace
}  // namespace dsg

using namespace dsg;

extern "C" int32_t dsg_validate_csr(const dsg_csr* g, int64_t n, int64_t m, int32_t* detail,
                                    void* stream) {
    if (detail) *detail = 0;
    if (!g || n < 0 || m < 0) return DSG_EINVAL;
    if (n > (int64_t)INT32_MAX - 1 || 2 * m > (int64_t)INT32_MAX) return DSG_EOVERFLOW;
    if (n > 0 && !g->row_ptr) return DSG_EINVAL;
    if (m > 0 && !g->col_idx) return DSG_EINVAL;
    if (n == 0) return m == 0 ? DSG_OK : DSG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int32_t* d_rule = nullptr;
    int32_t h_rule = kRuleNone;
    int32_t rc = DSG_OK;
    hipError_t e = hipMalloc((void**)&d_rule, sizeof(int32_t));
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? DSG_ENOMEM : DSG_EDEVICE;
    const unsigned grid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(2048, (n + kBlock - 1) / kBlock));
    const unsigned row_grid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(4096, (n + kWaves - 1) / kWaves));
    do {
        if ((e = hipMemcpyAsync(d_rule, &h_rule, sizeof(int32_t), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            break;
        k_check_rowptr<<<grid, kBlock, 0, s>>>(g->row_ptr, n, m, d_rule);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = hipMemcpyAsync(&h_rule, d_rule, sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            break;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
        if (h_rule != kRuleNone || m == 0) break;
        k_check_rows<<<row_grid, kBlock, 0, s>>>(g->row_ptr, g->col_idx, n, d_rule);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = hipMemcpyAsync(&h_rule, d_rule, sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            break;
        e = hipStreamSynchronize(s);
    } while (false);
    (void)hipFree(d_rule);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? DSG_ENOMEM : DSG_EDEVICE;
    if (h_rule != kRuleNone) {
        if (detail) *detail = h_rule;
        rc = DSG_EINVAL;
    }
    return rc;
}
