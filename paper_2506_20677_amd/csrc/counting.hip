// Counting sort pieces on gfx950 (Sec. III-F, Listing 2): the exclusive scan
// of the exact per-value histogram and, for keys without payload, the
// "expand" pass that writes every value as many times as it was counted.
// Also the tiny-input stable rank sort (the n <= 20 state of Sec. III-A) and
// fill helpers.
#include "common.hpp"
#include "kernels.hpp"

namespace ahs {

// ------------------------------------------------------------------ scan
// One workgroup: offsets[b] = sum of hist[0..b), offsets[nbins] = total.
constexpr int SCAN_THREADS = 1024;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_bins(const uint32_t* __restrict__ hist, uint32_t nbins,
                                                            uint32_t* __restrict__ offsets) {
  const uint32_t per = (nbins + SCAN_THREADS - 1) / SCAN_THREADS;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t local = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nbins) local += hist[b0 + i];
  __shared__ uint32_t sm[SCAN_THREADS / WAVE + 1];
  uint32_t total;
  uint32_t run = block_excl_scan<SCAN_THREADS>(local, sm, total);
  for (uint32_t i = 0; i < per; ++i) {
    if (b0 + i < nbins) {
      offsets[b0 + i] = run;
      run += hist[b0 + i];
    }
  }
  if (threadIdx.x == 0) offsets[nbins] = total;
}

hipError_t launch_scan_bins(const uint32_t* hist, uint32_t nbins, uint32_t* offsets, hipStream_t s) {
  k_scan_bins<<<1, SCAN_THREADS, 0, s>>>(hist, nbins, offsets);
  return hipGetLastError();
}

// ------------------------------------------------------------------ expand
// Keys-only counting sort output: position p holds min + b for the bin b
// with offsets[b] <= p < offsets[b+1].  Each block writes EXPAND_TILE
// consecutive positions; at each of 8 steps a thread writes 4 consecutive
// keys (one 16-byte store for u32 when aligned), so a wave stores 1 KiB
// contiguously.  The bin is found by binary search once and then advanced.
__device__ __forceinline__ uint32_t bin_of(const uint32_t* __restrict__ off, uint32_t nbins, uint64_t p) {
  // number of j in [1, nbins] with off[j] <= p
  uint32_t lo = 1, hi = nbins + 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((uint64_t)off[mid] <= p) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

template <int KK, bool VEC>
__global__ __launch_bounds__(EXPAND_THREADS) void k_expand(const uint32_t* __restrict__ off, uint32_t nbins,
                                                           typename KeyTraits<KK>::K kmin,
                                                           typename KeyTraits<KK>::K* __restrict__ out, uint64_t n) {
  using K = typename KeyTraits<KK>::K;
  const uint64_t base = (uint64_t)blockIdx.x * EXPAND_TILE;
  uint64_t p = base + (uint64_t)threadIdx.x * 4;
  if (p >= n) return;
  uint32_t b = bin_of(off, nbins, p);
  for (int step = 0; step < 8; ++step, p += EXPAND_THREADS * 4) {
    if (p >= n) break;
    if ((uint64_t)off[b + 1] <= p) {
      int tries = 0;
      while ((uint64_t)off[b + 1] <= p && tries < 8) { ++b; ++tries; }
      if ((uint64_t)off[b + 1] <= p) b = bin_of(off, nbins, p);
    }
    K v[4];
    uint32_t bb = b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      while ((uint64_t)off[bb + 1] <= p + j && bb + 1 < nbins) ++bb;
      v[j] = unmap_key<KK>((K)(kmin + (K)bb));
    }
    if (VEC && p + 4 <= n) {
      if constexpr (sizeof(K) == 4) {
        u32x4 w = {v[0], v[1], v[2], v[3]};
        *reinterpret_cast<u32x4*>(out + p) = w;
      } else {
        u64x2 w0 = {v[0], v[1]}, w1 = {v[2], v[3]};
        *reinterpret_cast<u64x2*>(out + p) = w0;
        *reinterpret_cast<u64x2*>(out + p + 2) = w1;
      }
    } else {
      for (int j = 0; j < 4; ++j)
        if (p + j < n) out[p + j] = v[j];
    }
  }
}

template <int KK>
static hipError_t expand_kk(const uint32_t* off, uint32_t nbins, uint64_t kmin, void* out, uint64_t n, hipStream_t s) {
  using K = typename KeyTraits<KK>::K;
  const int nb = (int)((n + EXPAND_TILE - 1) / EXPAND_TILE);
  if ((reinterpret_cast<uintptr_t>(out) & 15u) == 0)
    k_expand<KK, true><<<nb, EXPAND_THREADS, 0, s>>>(off, nbins, (K)kmin, (K*)out, n);
  else
    k_expand<KK, false><<<nb, EXPAND_THREADS, 0, s>>>(off, nbins, (K)kmin, (K*)out, n);
  return hipGetLastError();
}

hipError_t launch_expand(int kk, const uint32_t* offsets, uint32_t nbins, uint64_t kmin, void* out, uint64_t n,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  switch (kk) {
    case KK_U32: return expand_kk<KK_U32>(offsets, nbins, kmin, out, n, s);
    case KK_U64: return expand_kk<KK_U64>(offsets, nbins, kmin, out, n, s);
    case KK_F32: return expand_kk<KK_F32>(offsets, nbins, kmin, out, n, s);
    case KK_I32: return expand_kk<KK_I32>(offsets, nbins, kmin, out, n, s);
    case KK_F64: return expand_kk<KK_F64>(offsets, nbins, kmin, out, n, s);
    case KK_I64: return expand_kk<KK_I64>(offsets, nbins, kmin, out, n, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------ small sort
// Stable rank sort for n <= 1,024 in one workgroup: the rank of key i is the
// number of keys that are smaller, or equal and earlier.  This is the
// GPU form of the n <= 20 insertion-sort state: same unique stable output.
template <int KK, bool PAY>
__global__ __launch_bounds__(SMALL_SORT_MAX) void k_small_sort(const typename KeyTraits<KK>::K* __restrict__ src,
                                                               typename KeyTraits<KK>::K* __restrict__ dst,
                                                               const uint32_t* __restrict__ vsrc,
                                                               uint32_t* __restrict__ vdst, uint32_t n) {
  using K = typename KeyTraits<KK>::K;
  __shared__ K sk[SMALL_SORT_MAX];
  const uint32_t t = threadIdx.x;
  K k = 0;
  uint32_t v = 0;
  if (t < n) {
    k = map_key<KK>(src[t]);
    sk[t] = k;
    if (PAY) v = vsrc[t];
  }
  __syncthreads();
  if (t < n) {
    uint32_t r = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const K kj = sk[j];
      r += (kj < k) | ((kj == k) & (j < t));
    }
    dst[r] = unmap_key<KK>(k);
    if (PAY) vdst[r] = v;
  }
}

template <int KK>
static hipError_t small_kk(const void* src, void* dst, const uint32_t* vsrc, uint32_t* vdst, uint32_t n, hipStream_t s) {
  using K = typename KeyTraits<KK>::K;
  const int nt = (int)((n + 63) / 64 * 64);
  if (vsrc)
    k_small_sort<KK, true><<<1, nt, 0, s>>>((const K*)src, (K*)dst, vsrc, vdst, n);
  else
    k_small_sort<KK, false><<<1, nt, 0, s>>>((const K*)src, (K*)dst, nullptr, nullptr, n);
  return hipGetLastError();
}

hipError_t launch_small_sort(int kk, const void* src, void* dst, const uint32_t* vsrc, uint32_t* vdst, uint32_t n,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n > (uint32_t)SMALL_SORT_MAX) return hipErrorInvalidValue;
  switch (kk) {
    case KK_U32: return small_kk<KK_U32>(src, dst, vsrc, vdst, n, s);
    case KK_U64: return small_kk<KK_U64>(src, dst, vsrc, vdst, n, s);
    case KK_F32: return small_kk<KK_F32>(src, dst, vsrc, vdst, n, s);
    case KK_I32: return small_kk<KK_I32>(src, dst, vsrc, vdst, n, s);
    case KK_F64: return small_kk<KK_F64>(src, dst, vsrc, vdst, n, s);
    case KK_I64: return small_kk<KK_I64>(src, dst, vsrc, vdst, n, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------ fills
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ p, uint64_t count, T value) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256) p[i] = value;
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  uint64_t nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_fill<uint64_t><<<(int)nb, 256, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  uint64_t nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_fill<uint32_t><<<(int)nb, 256, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0 || src == dst) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

}  // namespace ahs
