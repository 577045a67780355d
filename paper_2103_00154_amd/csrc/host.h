// host.h - host-side argument checks and helpers shared by the translation
// units of libdsg.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "dsg.h"

namespace dsg {

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Sizes and eps for which every product of the method stays inside int64:
// 2(num+den)|E| and |V| den are the two sides of the failure test, and the
// int32 CSR needs n + 1 and 2m entries.
inline int32_t check_sizes(int64_t n, int64_t m, int64_t num, int64_t den) {
    if (n < 0 || m < 0 || den < 1 || num < 0) return DSG_EINVAL;
    if (n > (int64_t)INT32_MAX - 1) return DSG_EOVERFLOW;
    if (2 * (__int128)m > (__int128)INT32_MAX) return DSG_EOVERFLOW;
    if (num > INT64_MAX - den) return DSG_EOVERFLOW;
    const __int128 lim = (__int128)1 << 63;
    if ((__int128)2 * ((__int128)num + den) * m >= lim) return DSG_EOVERFLOW;
    if ((__int128)n * den >= lim) return DSG_EOVERFLOW;
    return DSG_OK;
}

// Upper bound on the number of passes: every pass of a valid input leaves
// fewer than |V| / (1 + eps) vertices, so log_{1+eps} n passes plus a margin
// suffice; with eps = 0 every pass still removes a vertex, so n passes do.
inline int32_t pass_bound(int64_t n, int64_t num, int64_t den) {
    if (n <= 1) return (int32_t)n;
    if (num == 0) return (int32_t)n;
    const double k = std::ceil(std::log((double)n) / std::log1p((double)num / (double)den));
    const double b = std::min((double)n, k + 2.0);
    return (int32_t)std::max(1.0, b);
}

inline int32_t map_hip(hipError_t e) {
    return e == hipErrorOutOfMemory ? DSG_ENOMEM : DSG_EDEVICE;
}

}  // namespace dsg
