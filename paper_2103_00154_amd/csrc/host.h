// host.h - host-side helpers shared by the translation units of libdsg.so:
// the argument checks of checks.h plus the HIP error mapping.
#pragma once

#include <hip/hip_runtime.h>

#include "checks.h"

namespace dsg {

inline int32_t map_hip(hipError_t e) {
    return e == hipErrorOutOfMemory ? DSG_ENOMEM : DSG_EDEVICE;
}

}  // namespace dsg
