// Fixed device scratch for ahs_sort_static: one file-scope array per GPU
// that the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is only a stand-in
// for the symbol); it uses the device address that hipGetSymbolAddress
// returns, taken once per device with that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "static_scratch.hpp"

static __device__ __align__(256) unsigned char scratch[ahs::STATIC_SCRATCH_BYTES];

namespace ahs {

namespace {
std::mutex g_mu;
void* g_addr[STATIC_SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t static_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= STATIC_SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace ahs
