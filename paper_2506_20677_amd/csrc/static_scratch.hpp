// Fixed per-device scratch behind ahs_sort_static (callers that cannot
// allocate device memory).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "ahs.h"

namespace ahs {

constexpr size_t STATIC_SCRATCH_BYTES = AHS_STATIC_SCRATCH_BYTES;
constexpr int STATIC_SCRATCH_MAX_DEVICES = 64;

// Device address of the scratch array on `device`, which must be the
// current device.  Looked up once per device, then cached.
hipError_t static_scratch_address(int device, void** out);

}  // namespace ahs
