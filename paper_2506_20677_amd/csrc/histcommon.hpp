// Streaming and LDS-counting helpers shared by the feature histograms and
// the batched sort's per-segment histograms and digit counts.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

// Compile-time tunables of the LDS histograms: lanes that must start in the
// first lane's bin for the wave to add that bin once; copies of the fused
// digit counters for 4- and 8-byte keys.
#ifndef AHS_HIST_GATE
#define AHS_HIST_GATE 8
#endif
#ifndef AHS_DIG_COPIES32
#define AHS_DIG_COPIES32 4
#endif
#ifndef AHS_DIG_COPIES64
#define AHS_DIG_COPIES64 2
#endif

namespace ahs {

// Streams the keys of [0, n) assigned to this thread with 16-byte loads
// (4 u32 or 2 u64 per load, UNROLL loads in flight), handling an unaligned
// head and the tail with scalar loads.  f(key) is called on raw bit patterns.
template <typename K, int UNROLL, typename F>
__device__ __forceinline__ void for_each_key(const K* __restrict__ keys, uint64_t n, uint64_t tid,
                                             uint64_t nthreads, F&& f) {
  constexpr int V = 16 / sizeof(K);
  const uintptr_t addr = reinterpret_cast<uintptr_t>(keys);
  uint64_t head = ((16u - (addr & 15u)) & 15u) / sizeof(K);
  if (head > n) head = n;
  for (uint64_t i = tid; i < head; i += nthreads) f(keys[i]);
  const uint64_t nvec = (n - head) / V;
  const u32x4* __restrict__ vp = reinterpret_cast<const u32x4*>(keys + head);
  uint64_t j = tid;
  for (; j + (UNROLL - 1) * nthreads < nvec; j += UNROLL * nthreads) {
    u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = vp[j + u * nthreads];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      if constexpr (sizeof(K) == 4) {
        f(v[u].x); f(v[u].y); f(v[u].z); f(v[u].w);
      } else {
        f((uint64_t)v[u].x | ((uint64_t)v[u].y << 32));
        f((uint64_t)v[u].z | ((uint64_t)v[u].w << 32));
      }
    }
  }
  for (; j < nvec; j += nthreads) {
    u32x4 v = vp[j];
    if constexpr (sizeof(K) == 4) {
      f(v.x); f(v.y); f(v.z); f(v.w);
    } else {
      f((uint64_t)v.x | ((uint64_t)v.y << 32));
      f((uint64_t)v.z | ((uint64_t)v.w << 32));
    }
  }
  for (uint64_t i = head + nvec * V + tid; i < n; i += nthreads) f(keys[i]);
}

// Same traversal, but hands the callback the V keys of one 16-byte load at
// once (g(keys, V)); head and tail keys come one at a time (g(keys, 1)).
template <typename K, int UNROLL, typename G>
__device__ __forceinline__ void for_each_group(const K* __restrict__ keys, uint64_t n, uint64_t tid,
                                               uint64_t nthreads, G&& g) {
  constexpr int V = 16 / sizeof(K);
  const uintptr_t addr = reinterpret_cast<uintptr_t>(keys);
  uint64_t head = ((16u - (addr & 15u)) & 15u) / sizeof(K);
  if (head > n) head = n;
  for (uint64_t i = tid; i < head; i += nthreads) {
    K one[V] = {keys[i]};
    g(one, 1);
  }
  const uint64_t nvec = (n - head) / V;
  const u32x4* __restrict__ vp = reinterpret_cast<const u32x4*>(keys + head);
  auto unpack = [](const u32x4& v, K (&kb)[V]) {
    if constexpr (sizeof(K) == 4) {
      kb[0] = v.x; kb[1] = v.y; kb[2] = v.z; kb[3] = v.w;
    } else {
      kb[0] = (uint64_t)v.x | ((uint64_t)v.y << 32);
      kb[1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
    }
  };
  uint64_t j = tid;
  for (; j + (UNROLL - 1) * nthreads < nvec; j += UNROLL * nthreads) {
    u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = vp[j + u * nthreads];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      K kb[V];
      unpack(v[u], kb);
      g(kb, V);
    }
  }
  for (; j < nvec; j += nthreads) {
    K kb[V];
    unpack(vp[j], kb);
    g(kb, V);
  }
  for (uint64_t i = head + nvec * V + tid; i < n; i += nthreads) {
    K one[V] = {keys[i]};
    g(one, 1);
  }
}

// True (in every lane) when at least a quarter of the wave's lanes start
// with bin c, the first active lane's first bin: sorted, nearly sorted and
// run-structured input, where one atomic per key would serialise on one LDS
// address.  Random input fails this one-ballot test and keeps the plain
// per-key path.
template <int V>
__device__ __forceinline__ bool wave_bin_dominant(const uint32_t (&b)[V], uint32_t c) {
  return popc64(__ballot(b[0] == c)) >= AHS_HIST_GATE;
}

// Takes the wave's keys of bin c out of `pend` and returns their number
// (the same in every lane).
template <int V>
__device__ __forceinline__ uint32_t take_wave_bin(const uint32_t (&b)[V], bool (&pend)[V], uint32_t c) {
  uint32_t tot = 0;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const bool e = pend[i] && b[i] == c;
    tot += popc64(__ballot(e));
    pend[i] = pend[i] && !e;
  }
  return tot;
}

// Counts m values (bins b[0..m) of this lane) into plain u32 LDS counters:
// one atomic per value, except that a dominant bin of the wave is added once
// by one lane.
template <int V>
__device__ __forceinline__ void lds_count_group(uint32_t* __restrict__ h, const uint32_t (&b)[V], int m) {
  const uint32_t c = __builtin_amdgcn_readfirstlane(b[0]);
  if (wave_bin_dominant<V>(b, c)) {
    bool pend[V];
#pragma unroll
    for (int i = 0; i < V; ++i) pend[i] = i < m;
    const uint32_t hit = take_wave_bin<V>(b, pend, c);
    if (mbcnt(__ballot(1)) == 0) atomicAdd(&h[c], hit);
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (pend[i]) atomicAdd(&h[b[i]], 1u);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (i < m) atomicAdd(&h[b[i]], 1u);
  }
}

}  // namespace ahs
