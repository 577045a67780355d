// host.h - host-side helpers shared by the translation units of libdsg.so:
// the argument checks of checks.h plus the HIP error mapping.
#pragma once

#include <hip/hip_runtime.h>

#include "checks.h"

namespace dsg {

inline int32_t map_hip(hipError_t e) {
    return e == hipErrorOutOfMemory ? DSG_ENOMEM : DSG_EDEVICE;
}

// dsg_peel_async with the workspace given (peel.hip).
int32_t peel_async(const dsg_csr* g, int64_t n, int64_t m, int64_t num, int64_t den,
                   int32_t* best_ids, int32_t* removed_at, dsg_batch_result* result,
                   const dsg_launch* launch, void* workspace, size_t ws_bytes, void* stream);

}  // namespace dsg
