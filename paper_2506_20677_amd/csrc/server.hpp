// Device pieces of the serving loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ahs {

struct CopyDesc {  // one contiguous copy of a multiple of 4 bytes, 4-byte aligned
  const void* src;
  void* dst;
  uint64_t bytes;
};

hipError_t launch_gather_copy(const CopyDesc* d_desc, uint32_t ndesc, uint64_t max_bytes, hipStream_t s);

}  // namespace ahs
