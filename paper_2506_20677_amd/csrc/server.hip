// Gather copy for the serving loop: moves every request's input (keys, and
// payload when present) into its batch's contiguous input region in one
// launch.  Grid row y takes descriptors y, y + gridDim.y, ...; x strides over
// each descriptor's bytes.
#include "common.hpp"
#include "server.hpp"

namespace ahs {

__global__ __launch_bounds__(256) void k_gather_copy(const CopyDesc* __restrict__ desc, uint32_t ndesc) {
  for (uint32_t y = blockIdx.y; y < ndesc; y += gridDim.y) {
  const CopyDesc d = desc[y];
  const uint64_t tid = (uint64_t)blockIdx.x * 256 + threadIdx.x, nthr = (uint64_t)gridDim.x * 256;
  const bool vec = ((reinterpret_cast<uintptr_t>(d.src) | reinterpret_cast<uintptr_t>(d.dst)) & 15u) == 0;
  if (vec) {
    const uint64_t nv = d.bytes / 16;
    const u32x4* __restrict__ s = static_cast<const u32x4*>(d.src);
    u32x4* __restrict__ t = static_cast<u32x4*>(d.dst);
    for (uint64_t i = tid; i < nv; i += nthr) t[i] = s[i];
    const uint64_t done = nv * 16;
    const uint32_t* __restrict__ s4 = static_cast<const uint32_t*>(d.src);
    uint32_t* __restrict__ t4 = static_cast<uint32_t*>(d.dst);
    for (uint64_t i = done / 4 + tid; i < d.bytes / 4; i += nthr) t4[i] = s4[i];
  } else {
    const uint32_t* __restrict__ s4 = static_cast<const uint32_t*>(d.src);
    uint32_t* __restrict__ t4 = static_cast<uint32_t*>(d.dst);
    for (uint64_t i = tid; i < d.bytes / 4; i += nthr) t4[i] = s4[i];
  }
  }
}

hipError_t launch_gather_copy(const CopyDesc* d_desc, uint32_t ndesc, uint64_t max_bytes, hipStream_t s) {
  if (ndesc == 0) return hipSuccess;
  const uint64_t chunks = (max_bytes + 256 * 16 * 4 - 1) / (256 * 16 * 4);
  const uint32_t gx = (uint32_t)(chunks < 1 ? 1 : (chunks > 1024 ? 1024 : chunks));
  const uint32_t gy = ndesc < 65535u ? ndesc : 65535u;  // the kernel strides over descriptors in y
  k_gather_copy<<<dim3(gx, gy), 256, 0, s>>>(d_desc, ndesc);
  return hipGetLastError();
}

}  // namespace ahs
