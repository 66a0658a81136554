// Device-side building blocks shared by the gfx950 kernels: key traits and
// the order-preserving float map, wave64 reductions, workgroup scans and
// agent-scope atomics for cross-XCD look-back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace ahs {

constexpr int WAVE = 64;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// K: the unsigned word a key is handled as.  FLT: IEEE keys (NaN possible,
// sign-magnitude bit map).  SGN: two's-complement keys (sign-bit flip).
// MAPPED: the stored bits are mapped on the first read and unmapped on the
// last write.
template <int KK> struct KeyTraits;
template <> struct KeyTraits<KK_U32> { using K = uint32_t; static constexpr bool FLT = false, SGN = false; };
template <> struct KeyTraits<KK_U64> { using K = uint64_t; static constexpr bool FLT = false, SGN = false; };
template <> struct KeyTraits<KK_F32> { using K = uint32_t; static constexpr bool FLT = true, SGN = false; };
template <> struct KeyTraits<KK_F64> { using K = uint64_t; static constexpr bool FLT = true, SGN = false; };
template <> struct KeyTraits<KK_I32> { using K = uint32_t; static constexpr bool FLT = false, SGN = true; };
template <> struct KeyTraits<KK_I64> { using K = uint64_t; static constexpr bool FLT = false, SGN = true; };
template <int KK> constexpr bool key_mapped = KeyTraits<KK>::FLT || KeyTraits<KK>::SGN;

// Order-preserving map of IEEE bit patterns onto unsigned integers: a set
// sign bit flips every bit, a clear one sets the sign bit.
__device__ __forceinline__ uint32_t fmap(uint32_t b) {
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint64_t fmap(uint64_t b) {
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ uint32_t funmap(uint32_t m) {
  return (m & 0x80000000u) ? (m & 0x7FFFFFFFu) : ~m;
}
__device__ __forceinline__ uint64_t funmap(uint64_t m) {
  return (m & 0x8000000000000000ull) ? (m & 0x7FFFFFFFFFFFFFFFull) : ~m;
}
__device__ __forceinline__ bool fnan(uint32_t b) { return (b & 0x7FFFFFFFu) > 0x7F800000u; }
__device__ __forceinline__ bool fnan(uint64_t b) {
  return (b & 0x7FFFFFFFFFFFFFFFull) > 0x7FF0000000000000ull;
}

// Order-preserving map of two's-complement keys onto unsigned integers (and
// its inverse): flip the sign bit.
template <typename K>
__device__ __forceinline__ K smap(K b) {
  return b ^ (K(1) << (8 * sizeof(K) - 1));
}

template <int KK>
__device__ __forceinline__ typename KeyTraits<KK>::K map_key(typename KeyTraits<KK>::K b) {
  if constexpr (KeyTraits<KK>::FLT) return fmap(b);
  else if constexpr (KeyTraits<KK>::SGN) return smap(b);
  else return b;
}
template <int KK>
__device__ __forceinline__ typename KeyTraits<KK>::K unmap_key(typename KeyTraits<KK>::K m) {
  if constexpr (KeyTraits<KK>::FLT) return funmap(m);
  else if constexpr (KeyTraits<KK>::SGN) return smap(m);
  else return m;
}

// ------------------------------------------------------------------ lanes
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint32_t popc64(uint64_t x) { return (uint32_t)__popcll(x); }

// Number of set bits of m below the calling lane (v_mbcnt pair).
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <typename T> __device__ __forceinline__ T shfl_xor(T v, int m) { return __shfl_xor(v, m, WAVE); }

template <typename T> __device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) { T o = shfl_xor(v, m); v = o < v ? o : v; }
  return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) { T o = shfl_xor(v, m); v = o > v ? o : v; }
  return v;
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
  return v;
}

// Inclusive scan across the 64 lanes of a wave.
template <typename T> __device__ __forceinline__ T wave_incl_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T o = __shfl_up(v, d, WAVE);
    if (l >= d) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread over a workgroup of NT threads;
// `smem` needs NT / 64 + 1 elements.  Returns the exclusive prefix and the total.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* smem, T& total) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE, l = lane_id();
  T inc = wave_incl_scan(v);
  if (l == WAVE - 1) smem[w] = inc;
  __syncthreads();
  if (w == 0) {
    T s = l < NW ? smem[l] : T(0);
    T si = wave_incl_scan(s);
    if (l < NW) smem[l] = si - s;
    if (l == NW - 1) smem[NW] = si;
  }
  __syncthreads();
  T res = smem[w] + inc - v;
  total = smem[NW];
  __syncthreads();
  return res;
}

// ------------------------------------------------------------------ atomics
// Agent (device) scope: coherent across the XCDs' separate L2 caches.
__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_agent(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ahs
